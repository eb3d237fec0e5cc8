// rg_brick.hip -- hydro update of complete 8x8x8-oct bricks on gfx950.
//
// Paper Sec. 3 (the rock/paper kernels): larger blocks of octs share their
// stencil so that fewer ghost cells are reconstructed redundantly; the
// paper's "paper" kernel sweeps a planar stencil through the block.  Here a
// brick is a Hilbert-aligned cube of 8^3 octs (16^3 cells) that all exist at
// one level; because an aligned sub-cube is a contiguous stretch of the
// Hilbert order, its 512 octs are consecutive in memory.  One workgroup of
// four wavefronts marches through the brick plane by plane along z:
//   - thread t owns interior column (x, y) = (t % 16, t / 16) and keeps the
//     primitive variables of planes z-1, z, z+1 of that column in registers;
//   - the current plane's primitive variables, the face states and the face
//     fluxes are exchanged through LDS;
//   - the ghost ring of the plane (two cells wide) is shared by all columns,
//     so a cell is reconstructed once per brick instead of once per oct.
// The arithmetic is the same per-cell/per-face code as the per-oct kernel
// (rg_math.hpp), evaluated on the same operands in the same order, so the
// two kernels produce identical bits.
//
// Bricks are used only where every neighbour oct of the brick exists at the
// same level or lies outside the domain; octs of other bricks (touching a
// coarse ghost, or partial) go to the per-oct kernel.
#include "rg_internal.hpp"
#include "rg_math.hpp"
#include "rg_brick.hpp"

namespace rg {
namespace {

// W: waves per SIMD the register allocation is sized for (the compiler
// spills beyond it); KU: see brick_body.  FP64 keeps the state in registers
// at two waves; the mixed form keeps it at three (the default: no second
// read of uold, fewer bricks sharing an XCD's L2) or reads it again at four
// (with KU it would spill).  Every variant gives the same bits.
template <typename R, int W, bool KU>
__global__ __launch_bounds__(BT, W) void k_hydro_brick(BrickArgs a)
{
    // two face buffers (one barrier per plane less) where the LDS still holds
    // as many workgroups as the registers allow: FP64 at two waves per SIMD
    // (76 KB), mixed at four (40 KB: its partial updates then need no LDS
    // slot) or three
    __shared__ BrickSmem<R, ((sizeof(R) == 8 && W == 2) || sizeof(R) == 4) ? 2 : 1> S;
    // consecutive bricks on one XCD: workgroups are dealt round-robin to the
    // eight XCDs, so give each XCD a contiguous Hilbert range of bricks
    const int64_t per_xcd = (a.nbricks + 7) / 8;
    const int64_t b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= a.nbricks) return;
    brick_body<R, KU>(a, a.bricks[b], b, S);
}

// Two bricks stacked along z per workgroup, swept as one column of 32
// planes: the two planes of ghost cells the sweep reconstructs at each end,
// and the slot table's setup, are shared by 32 planes instead of 16.  Used on
// a complete, periodic level with no split cell: every aligned brick of the
// level is then a brick of the schedule, and the first oct of brick (bx, by,
// bz) is the level's first oct plus 512 times the brick's Hilbert index
// among the level's bricks (a Hilbert-aligned cube is a contiguous stretch
// of the order, visited in the order of the coarser curve).  Pairs are taken
// in Morton order of (bx, by, bz / 2), each XCD a contiguous range of them.
// Same operands, same order per cell: the same bits as two single bricks.
template <typename R, int W, bool KU>
__global__ __launch_bounds__(BT, W) void k_hydro_brick_pair(BrickArgs a, int64_t first, int bl)
{
    __shared__ BrickSmem<R, ((sizeof(R) == 8 && W == 2) || sizeof(R) == 4) ? 2 : 1, 2> S;
    const int64_t npairs = a.nbricks / 2;
    const int64_t per_xcd = (npairs + 7) / 8;
    const int64_t p = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (p >= npairs) return;
    // bl: the level whose octs have the bricks' coordinates (2^(bl-1) per
    // side); the pair grid has m = bl - 1 bits in x and y, m - 1 in z
    const int m = bl - 1;
    int32_t bx = 0, by = 0, bz = 0;
    for (int t = 0; t < m; ++t) {
        bx |= static_cast<int32_t>((p >> (3 * t)) & 1) << t;
        by |= static_cast<int32_t>((p >> (3 * t + 1)) & 1) << t;
        if (t < m - 1) bz |= static_cast<int32_t>((p >> (3 * t + 2)) & 1) << t;
    }
    const uint64_t h0 = uint64_t(1) << (3 * (bl - 1));
    const int64_t lo = first + 512 * static_cast<int64_t>(oct_key(bx, by, 2 * bz, bl) - h0);
    const int64_t hi = first + 512 * static_cast<int64_t>(oct_key(bx, by, 2 * bz + 1, bl) - h0);
    brick_body<R, KU>(a, lo, p, S, hi);
}

}  // namespace

rg_status hydro_bricks(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                       const uint64_t *keys, const int32_t *bricks, int64_t nbricks, const double *dt, double dx,
                       double gamma, int outflow, int form, double cfl, double *dt_next, int waves, hipStream_t s,
                       int64_t pair_first, int pair_level)
{
    if (nbricks <= 0) return RG_OK;
    BrickArgs a;
    a.uold = uold;
    a.unew = unew;
    a.nbr27 = nbr27;
    a.son = son;
    a.keys = keys;
    a.bricks = bricks;
    a.nbricks = nbricks;
    a.dt = dt;
    a.dx = dx;
    a.gamma = gamma;
    a.outflow = outflow;
    a.cfl = cfl;
    a.dt_next = reinterpret_cast<unsigned long long *>(dt_next);
    a.hdr = current_sink();
    if (pair_level >= 5) {
        // the level's bricks two by two along z (see k_hydro_brick_pair)
        const int bl = pair_level - 3;
        RG_REQUIRE(nbricks == (int64_t(1) << (3 * (bl - 1))), "pairs need the level's every brick");
        const unsigned pgrid = static_cast<unsigned>(8 * ((nbricks / 2 + 7) / 8));
        if (form == RG_FP64) {
            if (waves == 0 || waves == 2)
                k_hydro_brick_pair<double, 2, true><<<pgrid, BT, 0, s>>>(a, pair_first, bl);
            else if (waves == 3)
                k_hydro_brick_pair<double, 3, false><<<pgrid, BT, 0, s>>>(a, pair_first, bl);
            else
                return fail(RG_ENOTSUP, "no FP64 brick kernel for %d waves per SIMD", waves);
        } else {
            if (waves == 4)
                k_hydro_brick_pair<float, 4, false><<<pgrid, BT, 0, s>>>(a, pair_first, bl);
            else if (waves == 0 || waves == 3)
                k_hydro_brick_pair<float, 3, true><<<pgrid, BT, 0, s>>>(a, pair_first, bl);
            else
                return fail(RG_ENOTSUP, "no mixed brick kernel for %d waves per SIMD", waves);
        }
        return launch_status("hydro brick pairs");
    }
    const unsigned grid = static_cast<unsigned>(8 * ((nbricks + 7) / 8));
    if (form == RG_FP64) {
        if (waves == 0 || waves == 2)
            k_hydro_brick<double, 2, true><<<grid, BT, 0, s>>>(a);
        else if (waves == 3)
            k_hydro_brick<double, 3, false><<<grid, BT, 0, s>>>(a);
        else
            return fail(RG_ENOTSUP, "no FP64 brick kernel for %d waves per SIMD", waves);
    } else {
        if (waves == 4)
            k_hydro_brick<float, 4, false><<<grid, BT, 0, s>>>(a);
        else if (waves == 0 || waves == 3)
            k_hydro_brick<float, 3, true><<<grid, BT, 0, s>>>(a);
        else
            return fail(RG_ENOTSUP, "no mixed brick kernel for %d waves per SIMD", waves);
    }
    return launch_status("hydro bricks");
}

}  // namespace rg

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

}  // namespace

rg_status hydro_bricks(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                       const uint64_t *keys, const int32_t *bricks, int64_t nbricks, const double *dt, double dx,
                       double gamma, int outflow, int form, double cfl, double *dt_next, int waves, hipStream_t s)
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

// rg_batch.hip -- many independent trees advanced by one graph launch.
//
// Every phase of a step (hash rebuild, neighbour lists, CFL dt per tree,
// hydro update of all trees and levels, coarse-fine corrections,
// restriction) is one persistent kernel that loops over a list of work
// items spanning all trees; the phases of all steps are captured once into
// a HIP graph, so a whole run is one hipGraphLaunch.  Each tree keeps its
// own time step (dt is a per-tree device slot).  The per-item work is the
// same device code as the single-tree kernels (rg_oct.hpp, rg_sib.hpp,
// rg_brick.hpp, rg_nbr.hpp), so a tree gives the same bits whether run alone
// or in a batch.
#include <algorithm>
#include <cstring>
#include <vector>

#include "rg_brick.hpp"
#include "rg_internal.hpp"
#include "rg_math.hpp"
#include "rg_nbr.hpp"
#include "rg_oct.hpp"
#include "rg_sib.hpp"

namespace rg {
namespace {

struct BTree {
    double *u[2];
    const uint64_t *keys;
    int32_t *nbr27;
    int32_t *father;
    uint32_t *son;
    double *corr;
    int64_t corr_base;
    const int32_t *list;     // the tree's schedule list
    HashHeader *hdr;
    uint64_t *hkeys;
    int32_t *hvals;
    uint64_t hmask;
    double gamma, cfl;
    int32_t lmin, lmax, bc, ghost;
    int64_t n_oct;
    int64_t level_begin[RG_MAX_LEVEL + 2];
};

// Work item: `tree`, a kind/level tag `a`, and a range [first, first+count)
// whose meaning depends on the phase.
struct Item {
    int32_t tree;
    int32_t a;
    int64_t first;
    int64_t count;
};

constexpr int kT = 256;   // threads of every batched kernel

// Items of a persistent loop: workgroups are dealt round-robin to the eight
// XCDs, so workgroup w serves a contiguous eighth of the item list (XCD
// w % 8), striding by the number of workgroups per XCD.  Neighbouring items
// (Hilbert-adjacent bricks sharing ghost cells) then meet in one L2.
struct ItemRange {
    int64_t begin, end, stride;
};

__device__ __forceinline__ ItemRange xcd_items(int64_t nitems)
{
    const int64_t per_xcd_wg = gridDim.x / 8;   // grid is a multiple of 8
    const int64_t x = blockIdx.x % 8, j = blockIdx.x / 8;
    const int64_t share = (nitems + 7) / 8;
    ItemRange r;
    r.begin = x * share + j;
    r.end = min(nitems, (x + 1) * share);
    r.stride = per_xcd_wg;
    return r;
}

__global__ void k_batch_dt_init(double *dt, int ntree)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntree) reinterpret_cast<unsigned long long *>(dt)[t] = 0x7ff0000000000000ull;
}

// cells [first, first+count) of one tree; one fold of the minimum per item
__global__ __launch_bounds__(kT) void k_batch_dt(const BTree *__restrict__ trees, const Item *__restrict__ items,
                                                  int64_t nitems, int parity, double *dt)
{
    __shared__ double s_min[kT / 64];
    const ItemRange r = xcd_items(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        const double *u = T.u[parity];
        double best = __longlong_as_double(0x7ff0000000000000ll);
        double nf = 0.0;
        for (int64_t cell = I.first + threadIdx.x; cell < I.first + I.count; cell += kT) {
            const int64_t o = cell >> 3;
            const int c = static_cast<int>(cell & 7);
            if ((T.son[o] >> c) & 1u) continue;
            int l = T.lmin;
            while (l < T.lmax && o >= T.level_begin[l + 1]) ++l;
            const double dx = ldexp(1.0, -l);
            double U[NV], W[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v] = u[NV * cell + v];
            prim64(U, T.gamma, W);
            const double cs = sqrt_pos(div_pos(T.gamma * W[4], W[0]));
            const double sp = ((fabs(W[1]) + fabs(W[2])) + fabs(W[3])) + 3.0 * cs;
            const double cd = T.cfl * (dx / sp);
            if (cd < best) best = cd;
            track_finite(nf, sp, U);
        }
        best = nonfinite_limit(best, nf);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            double o = __shfl_xor(best, off, 64);
            best = o < best ? o : best;
        }
        if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = s_min[0];
            for (int k = 1; k < kT / 64; ++k) m = s_min[k] < m ? s_min[k] : m;
            fold_min(reinterpret_cast<unsigned long long *>(dt + I.tree), m, T.hdr);
        }
        __syncthreads();
    }
}

// One item per workgroup, same XCD-contiguous dealing (grid = 8 ceil(n/8)).
__device__ __forceinline__ ItemRange xcd_item(int64_t nitems)
{
    const int64_t per_xcd = (nitems + 7) / 8;
    ItemRange r;
    r.begin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    r.end = r.begin < nitems ? r.begin + 1 : r.begin;
    r.stride = 1;
    return r;
}

// hydro update, item tag a = 4 level + kind.  Bricks (kind 0: the brick
// whose first oct is schedule list entry `first`) and oct groups (kind 1: up
// to G octs listed at [first, first+count) of the schedule list; kind 2: the
// octs first .. first+count-1) are separate kernels, so that each keeps the
// register allocation of its single-tree twin.
// With P the grid is persistent and loops over the items; without, each
// workgroup takes one item (no loop-carried registers).  FP64 bricks keep
// each column's state in registers (two waves per SIMD); mixed bricks read
// it again, at three waves: at four the loop spilled (72 scratch loads),
// and the 64-box graph took 38.0 ms against 35.2 ms at three.
template <typename R, bool P>
__global__ __launch_bounds__(BT, sizeof(R) == 8 ? 2 : 3) void k_batch_bricks(const BTree *__restrict__ trees,
                                                                            const Item *__restrict__ items,
                                                                            int64_t nitems, int parity,
                                                                            const double *dt, double *dt_next)
{
    __shared__ BrickSmem<R, 2> S;
    const ItemRange r = P ? xcd_items(nitems) : xcd_item(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        BrickArgs a;
        a.uold = T.u[parity];
        a.unew = T.u[parity ^ 1];
        a.nbr27 = T.nbr27;
        a.son = T.son;
        a.keys = T.keys;
        a.bricks = nullptr;
        a.nbricks = 0;
        a.dt = dt + I.tree;
        a.dx = ldexp(1.0, -(I.a >> 2));
        a.gamma = T.gamma;
        a.outflow = T.bc == RG_BC_OUTFLOW;
        a.cfl = T.cfl;
        a.dt_next = reinterpret_cast<unsigned long long *>(dt_next + I.tree);
        a.hdr = T.hdr;
        brick_body<R, sizeof(R) == 8>(a, T.list[I.first], I.first, S);
        __syncthreads();
    }
}

// registers as the compiler sees fit: a forced occupancy made the loop
// spill (up to 45 registers in the mixed form)
template <typename R, int G, bool P, bool GH>
__global__ __launch_bounds__(kT) void k_batch_octs(const BTree *__restrict__ trees, const Item *__restrict__ items,
                                                   int64_t nitems, int parity, const double *dt, double *dt_next)
{
    __shared__ Smem<R, G> S;
    const ItemRange r = P ? xcd_items(nitems) : xcd_item(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        const int level = I.a >> 2;
        LevelArgs a;
        a.list = (I.a & 3) == 1 ? T.list : nullptr;
        a.uold = T.u[parity];
        a.ucoarse = T.u[parity];
        a.unew = T.u[parity ^ 1];
        a.nbr27 = T.nbr27;
        a.son = T.son;
        a.corr = level > T.lmin ? T.corr : nullptr;
        a.corr_base = T.corr_base;
        a.corr_mode = 0;
        a.ghost = T.ghost;
        a.ucoarse2 = T.u[parity];
        a.oct_begin = I.first;
        a.oct_end = I.first + I.count;
        a.dt = dt + I.tree;
        a.dx = ldexp(1.0, -level);
        a.gamma = T.gamma;
        a.cfl = T.cfl;
        a.dt_next = reinterpret_cast<unsigned long long *>(dt_next + I.tree);
        a.hdr = T.hdr;
        hydro_group<R, G, kT, GH>(a, I.first, static_cast<int>(I.count), S);
        __syncthreads();
    }
}

// complete sibling groups: item = one group, `first` its entry in the tree's
// schedule list
template <typename R, bool P, bool GH>
__global__ __launch_bounds__(kT) void k_batch_groups(const BTree *__restrict__ trees, const Item *__restrict__ items,
                                                     int64_t nitems, int parity, const double *dt, double *dt_next)
{
    __shared__ SibSmem<R> S;
    const ItemRange r = P ? xcd_items(nitems) : xcd_item(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        const int level = I.a >> 2;
        LevelArgs a;
        a.list = T.list;
        a.uold = T.u[parity];
        a.ucoarse = T.u[parity];
        a.unew = T.u[parity ^ 1];
        a.nbr27 = T.nbr27;
        a.son = T.son;
        a.corr = level > T.lmin ? T.corr : nullptr;
        a.corr_base = T.corr_base;
        a.corr_mode = 0;
        a.ghost = T.ghost;
        a.ucoarse2 = T.u[parity];
        a.oct_begin = I.first;
        a.oct_end = I.first + 1;
        a.dt = dt + I.tree;
        a.dx = ldexp(1.0, -level);
        a.gamma = T.gamma;
        a.cfl = T.cfl;
        a.dt_next = reinterpret_cast<unsigned long long *>(dt_next + I.tree);
        a.hdr = T.hdr;
        hydro_sib<R, kT, GH>(a, T.father, T.list[I.first], S);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kT) void k_batch_corr(const BTree *__restrict__ trees, const Item *__restrict__ items,
                                                    int64_t nitems, int parity, int side)
{
    const int ax = side >> 1, hi = side & 1;
    const int slot = (ax == 0 ? (hi ? 2 : 0) : 1) + 3 * (ax == 1 ? (hi ? 2 : 0) : 1) + 9 * (ax == 2 ? (hi ? 2 : 0) : 1);
    const ItemRange r = xcd_items(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        double *unew = T.u[parity ^ 1];
        for (int64_t k = threadIdx.x; k < I.count * NV; k += kT) {
            const int64_t o = I.first + k / NV;
            const int v = static_cast<int>(k % NV);
            const int32_t e = T.nbr27[27 * o + slot];
            if (!(e < 0 && e != RG_NBR_OUTSIDE)) continue;
            const int64_t C = -1 - int64_t(e);
            unew[NV * C + v] = unew[NV * C + v] + T.corr[30 * (o - T.corr_base) + NV * side + v];
        }
    }
}

// CFL limit of the coarse cells the corrections changed (every coarse face
// neighbour of the item's octs), folded into the tree's next time step
__global__ __launch_bounds__(kT) void k_batch_corr_dt(const BTree *__restrict__ trees,
                                                       const Item *__restrict__ items, int64_t nitems, int parity,
                                                       double *dt_next)
{
    __shared__ double s_min[kT / 64];
    const ItemRange r = xcd_items(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        const double *u = T.u[parity ^ 1];
        double best = __longlong_as_double(0x7ff0000000000000ll);
        double nf = 0.0;
        for (int64_t k = threadIdx.x; k < I.count * 6; k += kT) {
            const int64_t o = I.first + k / 6;
            const int side = static_cast<int>(k % 6);
            const int ax = side >> 1, hi = side & 1;
            const int slot = (ax == 0 ? (hi ? 2 : 0) : 1) + 3 * (ax == 1 ? (hi ? 2 : 0) : 1) +
                             9 * (ax == 2 ? (hi ? 2 : 0) : 1);
            const int32_t e = T.nbr27[27 * o + slot];
            if (!(e < 0 && e != RG_NBR_OUTSIDE)) continue;
            const int64_t C = -1 - int64_t(e);
            int l = T.lmin;
            while (l < T.lmax && o >= T.level_begin[l + 1]) ++l;
            const double dx = ldexp(1.0, -(l - 1));
            double U[NV], W[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v] = u[NV * C + v];
            prim64(U, T.gamma, W);
            const double cs = sqrt_pos(div_pos(T.gamma * W[4], W[0]));
            const double sp = ((fabs(W[1]) + fabs(W[2])) + fabs(W[3])) + 3.0 * cs;
            const double cd = T.cfl * (dx / sp);
            if (cd < best) best = cd;
            track_finite(nf, sp, U);
        }
        best = nonfinite_limit(best, nf);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            double o = __shfl_xor(best, off, 64);
            best = o < best ? o : best;
        }
        if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = s_min[0];
            for (int k = 1; k < kT / 64; ++k) m = s_min[k] < m ? s_min[k] : m;
            fold_min(reinterpret_cast<unsigned long long *>(dt_next + I.tree), m, T.hdr);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kT) void k_batch_restrict(const BTree *__restrict__ trees,
                                                        const Item *__restrict__ items, int64_t nitems, int parity)
{
    const ItemRange r = xcd_items(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        double *u = T.u[parity ^ 1];
        for (int64_t k = threadIdx.x; k < I.count * NV; k += kT) {
            const int64_t o = I.first + k / NV;
            const int v = static_cast<int>(k % NV);
            const double *c = u + 8 * NV * o + v;
            const double sum = ((c[0] + c[5]) + (c[10] + c[15])) + ((c[20] + c[25]) + (c[30] + c[35]));
            u[NV * int64_t(T.father[o]) + v] = 0.125 * sum;
        }
    }
}

// tree bookkeeping: son masks and hash slots cleared, keys inserted
__global__ __launch_bounds__(kT) void k_batch_clear(const BTree *__restrict__ trees, const Item *__restrict__ items,
                                                     int64_t nitems)
{
    const ItemRange r = xcd_items(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        if (I.a == 0) {
            for (int64_t k = threadIdx.x; k < I.count; k += kT) T.hkeys[I.first + k] = 0;
            if (I.first == 0 && threadIdx.x == 0) {
                T.hdr->cap = T.hmask + 1;
                T.hdr->n = T.n_oct;
                T.hdr->err = 0;
                T.hdr->bad = -1;
            }
        } else {
            for (int64_t k = threadIdx.x; k < I.count; k += kT) T.son[I.first + k] = 0u;
        }
    }
}

__global__ __launch_bounds__(kT) void k_batch_insert(const BTree *__restrict__ trees, const Item *__restrict__ items,
                                                      int64_t nitems)
{
    const ItemRange r = xcd_items(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        for (int64_t k = threadIdx.x; k < I.count; k += kT) hash_insert_one(T.hdr, T.hkeys, T.hvals, T.hmask,
                                                                             T.keys[I.first + k], I.first + k);
    }
}

__global__ __launch_bounds__(kT) void k_batch_nbr(const BTree *__restrict__ trees, const Item *__restrict__ items,
                                                   int64_t nitems)
{
    __shared__ union {
        NbrGroup grp;
        NbrBrick brick;
    } S;
    const ItemRange r = xcd_items(nitems);
    for (int64_t it = r.begin; it < r.end; it += r.stride) {
        const Item I = items[it];
        const BTree &T = trees[I.tree];
        const NbrTable tab{T.keys, T.hdr, T.hkeys, T.hvals, T.hmask, T.nbr27, T.father, T.son, T.lmin, T.bc,
                           RG_MAX_LEVEL + 1};
        if (I.a == 0)
            nbr_brick_body(tab, T.list[I.first], S.brick);
        else
            nbr_octs_body(tab, T.list, I.first, static_cast<int>(I.count), S.grp);
        __syncthreads();
    }
}

struct Phase {
    Item *d_items = nullptr;
    int64_t n = 0;
};

}  // namespace
}  // namespace rg

using namespace rg;

struct rg_batch {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *d_mem = nullptr;   // tree table and item lists
    int ntree = 0;
    int nsteps = 0;
};

namespace {

// compute units of the current device (256 on MI355X)
int64_t device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

// a persistent grid: as many workgroups as fit on the device at once (a
// multiple of 8, one share per XCD), at most one per item
int persistent_grid(const void *kernel, int threads, int64_t nitems)
{
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1) per = 1;
    const int64_t want = std::min<int64_t>(device_cus() * per, nitems);
    return static_cast<int>(std::max<int64_t>(8, (want + 7) / 8 * 8));
}

unsigned one_shot_grid(int64_t nitems) { return static_cast<unsigned>(8 * ((nitems + 7) / 8)); }

template <typename R>
rg_status launch_bricks(bool persistent, const BTree *trees, const Phase &p, int parity, const double *dt,
                        double *dt_next, hipStream_t s)
{
    if (p.n == 0) return RG_OK;
    if (persistent) {
        const int grid = persistent_grid(reinterpret_cast<const void *>(&k_batch_bricks<R, true>), BT, p.n);
        k_batch_bricks<R, true><<<grid, BT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
    } else {
        k_batch_bricks<R, false><<<one_shot_grid(p.n), BT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
    }
    return launch_status("batched bricks");
}

template <typename R, int G, bool GH>
rg_status launch_octs(bool persistent, const BTree *trees, const Phase &p, int parity, const double *dt,
                      double *dt_next, hipStream_t s)
{
    if (p.n == 0) return RG_OK;
    if (persistent) {
        const int grid = persistent_grid(reinterpret_cast<const void *>(&k_batch_octs<R, G, true, GH>), kT, p.n);
        k_batch_octs<R, G, true, GH><<<grid, kT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
    } else {
        k_batch_octs<R, G, false, GH><<<one_shot_grid(p.n), kT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
    }
    return launch_status("batched oct groups");
}

template <typename R>
rg_status launch_octs_g(int g, bool gh, bool persistent, const BTree *trees, const Phase &p, int parity,
                        const double *dt, double *dt_next, hipStream_t s)
{
    if (gh) {
        if (g == 2) return launch_octs<R, 2, true>(persistent, trees, p, parity, dt, dt_next, s);
        if (g == 8) return launch_octs<R, 8, true>(persistent, trees, p, parity, dt, dt_next, s);
        return launch_octs<R, 4, true>(persistent, trees, p, parity, dt, dt_next, s);
    }
    if (g == 2) return launch_octs<R, 2, false>(persistent, trees, p, parity, dt, dt_next, s);
    if (g == 8) return launch_octs<R, 8, false>(persistent, trees, p, parity, dt, dt_next, s);
    return launch_octs<R, 4, false>(persistent, trees, p, parity, dt, dt_next, s);
}

template <typename R>
rg_status launch_groups(bool gh, bool persistent, const BTree *trees, const Phase &p, int parity, const double *dt,
                        double *dt_next, hipStream_t s)
{
    if (p.n == 0) return RG_OK;
    if (persistent) {
        if (gh) {
            const int grid = persistent_grid(reinterpret_cast<const void *>(&k_batch_groups<R, true, true>), kT, p.n);
            k_batch_groups<R, true, true><<<grid, kT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
        } else {
            const int grid = persistent_grid(reinterpret_cast<const void *>(&k_batch_groups<R, true, false>), kT, p.n);
            k_batch_groups<R, true, false><<<grid, kT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
        }
    } else if (gh) {
        k_batch_groups<R, false, true><<<one_shot_grid(p.n), kT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
    } else {
        k_batch_groups<R, false, false><<<one_shot_grid(p.n), kT, 0, s>>>(trees, p.d_items, p.n, parity, dt, dt_next);
    }
    return launch_status("batched sibling groups");
}

unsigned small_grid(int64_t n)
{
    const int64_t want = std::min<int64_t>(n, 4 * device_cus());
    return static_cast<unsigned>(std::max<int64_t>(8, (want + 7) / 8 * 8));
}

void chunk(std::vector<Item> &v, int tree, int a, int64_t first, int64_t count, int64_t size)
{
    for (int64_t k = 0; k < count; k += size) v.push_back(Item{tree, a, first + k, std::min(size, count - k)});
}

}  // namespace

extern "C" {

rg_status rg_batch_create(const rg_batch_tree *trees, int ntree, int form, int nsteps, unsigned flags,
                          const rg_tuning *tune, double *d_dt, void *stream, rg_batch **out)
{
    RG_REQUIRE(trees && ntree > 0 && nsteps > 0 && d_dt && out, "bad arguments");
    RG_REQUIRE(form == RG_FP64 || form == RG_MIXED, "bad form %d", form);
    RG_REQUIRE((flags & ~RG_STEP_REBUILD) == 0, "unsupported flags %u", flags);
    const int g = tune && tune->octs_per_group ? tune->octs_per_group : 4;
    RG_REQUIRE(g == 2 || g == 4 || g == 8, "batched kernel has no %d-oct groups", g);
    const bool bricks = !(tune && tune->no_bricks);
    const bool groups = bricks && !(tune && tune->no_groups);
    const bool persistent = tune && tune->persistent;
    bool gh = false;   // some tree interpolates its coarse ghosts
    for (int t = 0; t < ntree; ++t) gh = gh || (trees[t].tree && trees[t].tree->ghost == RG_GHOST_LINEAR);
    *out = nullptr;
    hipStream_t s = as_stream(stream);

    std::vector<BTree> bt(ntree);
    std::vector<Item> it_bricks, it_octs, it_groups, it_dt, it_corr, it_clear, it_insert, it_nbr;
    std::vector<std::vector<Item>> it_restrict;
    int maxdepth = 0;
    for (int t = 0; t < ntree; ++t) {
        const rg_tree *T = trees[t].tree;
        RG_REQUIRE(T && T->sched && T->sched->d_list, "tree %d has no schedule", t);
        RG_REQUIRE(trees[t].d_u0 && trees[t].d_u1 && trees[t].d_u0 != trees[t].d_u1, "tree %d state buffers", t);
        RG_REQUIRE(T->n_oct > 0 && T->lmin >= 1 && T->lmax >= T->lmin && T->lmax <= RG_MAX_LEVEL, "tree %d levels", t);
        RG_REQUIRE(T->level_begin[T->lmin] == 0 && T->level_begin[T->lmax + 1] == T->n_oct, "tree %d level ranges", t);
        RG_REQUIRE(T->lmin == T->lmax || T->d_corr, "tree %d needs a correction buffer", t);
        RG_REQUIRE(T->ghost == RG_GHOST_INJECT || T->ghost == RG_GHOST_LINEAR, "tree %d ghost mode", t);
        RG_REQUIRE(T->d_keys && T->d_hash_ws && T->d_nbr27 && T->d_father_cell && T->d_son_mask, "tree %d buffers", t);
        RG_REQUIRE(trees[t].gamma > 1 && trees[t].cfl > 0, "tree %d gamma/cfl", t);
        const rg_schedule *sc = T->sched;
        const uint64_t cap = hash_capacity(T->n_oct);
        HashView h = hash_view(T->d_hash_ws, cap);
        BTree &b = bt[t];
        b.u[0] = trees[t].d_u0;
        b.u[1] = trees[t].d_u1;
        b.keys = T->d_keys;
        b.nbr27 = T->d_nbr27;
        b.father = T->d_father_cell;
        b.son = T->d_son_mask;
        b.corr = T->d_corr;
        b.corr_base = T->level_begin[T->lmin + 1];
        b.list = sc->d_list;
        b.hdr = h.hdr;
        b.hkeys = h.keys;
        b.hvals = h.vals;
        b.hmask = h.mask;
        b.gamma = trees[t].gamma;
        b.cfl = trees[t].cfl;
        b.lmin = T->lmin;
        b.lmax = T->lmax;
        b.bc = T->bc;
        b.ghost = T->ghost;
        b.n_oct = T->n_oct;
        for (int l = 0; l < RG_MAX_LEVEL + 2; ++l) b.level_begin[l] = T->level_begin[l];

        for (int l = T->lmin; l <= T->lmax; ++l) {
            if (groups) {
                for (int64_t k = 0; k < sc->brick_count[l]; ++k)
                    it_bricks.push_back(Item{t, 4 * l, sc->brick_begin[l] + k, 1});
                for (int64_t k = 0; k < sc->group_count[l]; ++k)
                    it_groups.push_back(Item{t, 4 * l + 3, sc->group_begin[l] + k, 1});
                chunk(it_octs, t, 4 * l + 1, sc->single_begin[l], sc->single_count[l], g);
            } else if (bricks) {
                for (int64_t k = 0; k < sc->brick_count[l]; ++k)
                    it_bricks.push_back(Item{t, 4 * l, sc->brick_begin[l] + k, 1});
                chunk(it_octs, t, 4 * l + 1, sc->rest_begin[l], sc->rest_count[l], g);
            } else {
                chunk(it_octs, t, 4 * l + 2, T->level_begin[l], T->level_begin[l + 1] - T->level_begin[l], g);
            }
        }
        chunk(it_dt, t, 0, 0, 8 * T->n_oct, 4096);
        if (T->lmax > T->lmin) chunk(it_corr, t, 0, b.corr_base, T->n_oct - b.corr_base, 1024);
        maxdepth = std::max(maxdepth, T->lmax - T->lmin);
        chunk(it_clear, t, 0, 0, static_cast<int64_t>(cap), 65536);
        chunk(it_clear, t, 1, 0, T->n_oct, 65536);
        chunk(it_insert, t, 0, 0, T->n_oct, 4096);
        for (int64_t k = 0; k < sc->nbr_brick_count; ++k) it_nbr.push_back(Item{t, 0, sc->nbr_brick_begin + k, 1});
        chunk(it_nbr, t, 1, sc->nbr_rest_begin, sc->nbr_rest_count, kNbrOcts);
    }
    it_restrict.resize(maxdepth);
    for (int k = 0; k < maxdepth; ++k)
        for (int t = 0; t < ntree; ++t) {
            const rg_tree *T = trees[t].tree;
            const int L = T->lmax - k;
            if (L > T->lmin)
                chunk(it_restrict[k], t, L, T->level_begin[L], T->level_begin[L + 1] - T->level_begin[L], 1024);
        }
    // one device allocation: tree table then item lists
    std::vector<const std::vector<Item> *> lists = {&it_bricks, &it_octs, &it_dt, &it_corr,
                                                      &it_clear, &it_insert, &it_nbr, &it_groups};
    for (auto &v : it_restrict) lists.push_back(&v);
    size_t bytes = (sizeof(BTree) * ntree + 255) & ~size_t(255);
    for (auto *v : lists) bytes += (v->size() * sizeof(Item) + 255) & ~size_t(255);
    rg_batch *B = new rg_batch();
    B->ntree = ntree;
    B->nsteps = nsteps;
    hipError_t e = hipMalloc(&B->d_mem, bytes);
    if (e != hipSuccess) {
        delete B;
        return fail(RG_EHIP, "batch table: %s", hipGetErrorString(e));
    }
    std::vector<char> host(bytes, 0);
    size_t off = 0;
    std::memcpy(host.data(), bt.data(), sizeof(BTree) * ntree);
    const BTree *d_trees = reinterpret_cast<const BTree *>(B->d_mem);
    off = (sizeof(BTree) * ntree + 255) & ~size_t(255);
    std::vector<Phase> phases;
    for (auto *v : lists) {
        Phase p;
        p.d_items = reinterpret_cast<Item *>(static_cast<char *>(B->d_mem) + off);
        p.n = static_cast<int64_t>(v->size());
        if (!v->empty()) std::memcpy(host.data() + off, v->data(), v->size() * sizeof(Item));
        off += (v->size() * sizeof(Item) + 255) & ~size_t(255);
        phases.push_back(p);
    }
    e = hipMemcpyAsync(B->d_mem, host.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(B->d_mem);
        delete B;
        return fail(RG_EHIP, "batch upload: %s", hipGetErrorString(e));
    }
    enum { P_BRICKS, P_OCTS, P_DT, P_CORR, P_CLEAR, P_INSERT, P_NBR, P_GROUPS, P_RESTRICT };
    const Phase &ph_bricks = phases[P_BRICKS], &ph_octs = phases[P_OCTS], &ph_dt = phases[P_DT],
                &ph_corr = phases[P_CORR], &ph_clear = phases[P_CLEAR], &ph_insert = phases[P_INSERT],
                &ph_nbr = phases[P_NBR], &ph_groups = phases[P_GROUPS];
    const unsigned g_dt = small_grid(ph_dt.n), g_corr = small_grid(ph_corr.n), g_clear = small_grid(ph_clear.n),
                   g_insert = small_grid(ph_insert.n), g_nbr = small_grid(ph_nbr.n);
    std::vector<unsigned> g_restrict(maxdepth);
    for (int k = 0; k < maxdepth; ++k) g_restrict[k] = small_grid(phases[P_RESTRICT + k].n);
    // warm the occupancy queries outside the capture
    (void)persistent_grid(reinterpret_cast<const void *>(&k_batch_bricks<double, true>), BT, 1);

    // capture all steps into one graph; within a step the bricks and the
    // other octs (sibling groups, then single octs; disjoint outputs) are two
    // branches that may run concurrently
    hipStream_t cs = nullptr, cs2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    auto release = [&]() {
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (cs2) (void)hipStreamDestroy(cs2);
        if (cs) (void)hipStreamDestroy(cs);
    };
    if (e != hipSuccess) {
        release();
        (void)hipFree(B->d_mem);
        delete B;
        return fail(RG_EHIP, "graph capture: %s", hipGetErrorString(e));
    }
    rg_status st = RG_OK;
    for (int step = 0; step < nsteps && st == RG_OK; ++step) {
        const int parity = step & 1;
        // row `step` of d_dt is this step's time step (a pass over the state
        // for the first step, folded into the previous step otherwise); the
        // update folds the next one into row step+1
        double *dt = d_dt + static_cast<int64_t>(step) * ntree;
        double *dt_next = dt + ntree;
        if (flags & RG_STEP_REBUILD) {
            k_batch_clear<<<g_clear, kT, 0, cs>>>(d_trees, ph_clear.d_items, ph_clear.n);
            k_batch_insert<<<g_insert, kT, 0, cs>>>(d_trees, ph_insert.d_items, ph_insert.n);
            k_batch_nbr<<<g_nbr, kT, 0, cs>>>(d_trees, ph_nbr.d_items, ph_nbr.n);
        }
        if (step == 0) {
            k_batch_dt_init<<<(ntree + 255) / 256, 256, 0, cs>>>(dt, ntree);
            k_batch_dt<<<g_dt, kT, 0, cs>>>(d_trees, ph_dt.d_items, ph_dt.n, parity, dt);
        }
        k_batch_dt_init<<<(ntree + 255) / 256, 256, 0, cs>>>(dt_next, ntree);
        const bool fork = ph_bricks.n > 0 && (ph_octs.n > 0 || ph_groups.n > 0);
        if (fork) {
            e = hipEventRecord(ev_fork, cs);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs2, ev_fork, 0);
            if (e != hipSuccess) {
                st = fail(RG_EHIP, "graph fork: %s", hipGetErrorString(e));
                break;
            }
        }
        if (form == RG_FP64)
            st = launch_bricks<double>(persistent, d_trees, ph_bricks, parity, dt, dt_next, cs);
        else
            st = launch_bricks<float>(persistent, d_trees, ph_bricks, parity, dt, dt_next, cs);
        if (st != RG_OK) break;
        hipStream_t so = fork ? cs2 : cs;
        if (form == RG_FP64)
            st = launch_groups<double>(gh, persistent, d_trees, ph_groups, parity, dt, dt_next, so);
        else
            st = launch_groups<float>(gh, persistent, d_trees, ph_groups, parity, dt, dt_next, so);
        if (st != RG_OK) break;
        if (form == RG_FP64)
            st = launch_octs_g<double>(g, gh, persistent, d_trees, ph_octs, parity, dt, dt_next, so);
        else
            st = launch_octs_g<float>(g, gh, persistent, d_trees, ph_octs, parity, dt, dt_next, so);
        if (st != RG_OK) break;
        if (fork) {
            e = hipEventRecord(ev_join, cs2);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev_join, 0);
            if (e != hipSuccess) {
                st = fail(RG_EHIP, "graph join: %s", hipGetErrorString(e));
                break;
            }
        }
        if (ph_corr.n) {
            for (int side = 0; side < 6; ++side)
                k_batch_corr<<<g_corr, kT, 0, cs>>>(d_trees, ph_corr.d_items, ph_corr.n, parity, side);
            k_batch_corr_dt<<<g_corr, kT, 0, cs>>>(d_trees, ph_corr.d_items, ph_corr.n, parity, dt_next);
        }
        for (int k = 0; k < maxdepth; ++k) {
            const Phase &p = phases[P_RESTRICT + k];
            if (p.n) k_batch_restrict<<<g_restrict[k], kT, 0, cs>>>(d_trees, p.d_items, p.n, parity);
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    release();
    if (st == RG_OK && ec != hipSuccess) st = fail(RG_EHIP, "end capture: %s", hipGetErrorString(ec));
    if (st == RG_OK) st = launch_status("batch capture");
    if (st == RG_OK) {
        e = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = fail(RG_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    B->graph = graph;
    if (st != RG_OK) {
        if (B->exec) (void)hipGraphExecDestroy(B->exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipFree(B->d_mem);
        delete B;
        return st;
    }
    *out = B;
    return RG_OK;
}

rg_status rg_batch_run(rg_batch *b, void *stream)
{
    RG_REQUIRE(b && b->exec, "null batch");
    hipError_t e = hipGraphLaunch(b->exec, as_stream(stream));
    if (e != hipSuccess) return fail(RG_EHIP, "graph launch: %s", hipGetErrorString(e));
    return RG_OK;
}

rg_status rg_batch_destroy(rg_batch *b)
{
    if (!b) return RG_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_mem) (void)hipFree(b->d_mem);
    delete b;
    return RG_OK;
}

}  // extern "C"

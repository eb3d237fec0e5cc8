// rg_hydro.hip -- per-level hydrodynamics update on gfx950.
//
// Paper Sec. 3: a second-order Godunov MUSCL-Hancock predictor-corrector
// with an HLLC Riemann solver; each oct is updated from a local stencil of
// 6x6x6 cells (the oct plus two ghost cells per side) holding uold:
// conservative -> primitive, face-centred states, Riemann fluxes, update into
// unew.  Table 1 rows "compute dt" and "hydro - upload" are rg_cfl_dt and
// rg_restrict_level.
//
// Kernel shape: a workgroup serves G consecutive octs of one level (Hilbert
// order keeps them spatially close).  Every phase is a flat loop over
// (oct, item) pairs so the 64-wide wavefronts stay busy:
//   A gather + primitive variables for the 80 stencil cells an oct needs
//   B slopes, predictor, face states for the 32 cells touching its faces
//   C HLLC on the 36 faces of its 8 cells
//   D conservative update of its 40 (cell, variable) values
//   E fluxes owed to coarse neighbours (6 sides x 5 variables)
// All intermediate data stay in LDS; HBM sees uold (stencil reads, mostly
// L2 hits between neighbouring octs), the neighbour list and unew.
#include "rg_internal.hpp"
#include "rg_math.hpp"
#include "rg_oct.hpp"
#include "rg_sib.hpp"

namespace rg {
namespace {

template <typename R, int G, int NT, bool GH>
__global__ __launch_bounds__(NT) void k_hydro_level(LevelArgs a)
{
    __shared__ Smem<R, G> S;
    const int64_t first = a.oct_begin + int64_t(blockIdx.x) * G;
    const int64_t left = a.oct_end - first;
    const int count = left < G ? static_cast<int>(left) : G;
    hydro_group<R, G, NT, GH>(a, first, count, S);
}

// one complete sibling group per workgroup: list[oct_begin + block] is the
// group's first oct
template <typename R, int NT, bool GH>
__global__ __launch_bounds__(NT) void k_hydro_sib(LevelArgs a, const int32_t *__restrict__ father)
{
    __shared__ SibSmem<R> S;
    hydro_sib<R, NT, GH>(a, father, a.list[a.oct_begin + blockIdx.x], S);
}

// ---------------------------------------------------------------------------
// CFL time step, corrections, restriction
// ---------------------------------------------------------------------------

struct DtArgs {
    const double *u;
    const uint32_t *son;
    int64_t begin[RG_MAX_LEVEL + 2];
    int lmin, lmax;
    double gamma, cfl;
    int64_t n_cell;
    unsigned long long *dt_bits;
    HashHeader *hdr;   // device-side errors (non-finite state)
    int sub;   // subcycled: each limit scaled by 2^(l - lmin), the ratio of the coarse step to level l's
};

__global__ void k_set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

// Grid-stride over cells: a bounded grid keeps the final atomics few.
__global__ __launch_bounds__(256) void k_cfl_dt(DtArgs a)
{
    double best = __longlong_as_double(0x7ff0000000000000ll);   // +inf
    double nf = 0.0;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t cell = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; cell < a.n_cell; cell += stride) {
        const int64_t o = cell >> 3;
        const int c = static_cast<int>(cell & 7);
        if ((a.son[o] >> c) & 1u) continue;
        int l = a.lmin;
        while (l < a.lmax && o >= a.begin[l + 1]) ++l;
        const double dx = ldexp(1.0, -l);
        double U[NV], W[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = a.u[NV * cell + v];
        prim64(U, a.gamma, W);
        const double cs = sqrt_pos(div_pos(a.gamma * W[4], W[0]));
        const double sp = ((fabs(W[1]) + fabs(W[2])) + fabs(W[3])) + 3.0 * cs;
        const double d = a.sub ? ldexp(dx / sp, l - a.lmin) : dx / sp;
        // cfl * min(d) == min(cfl * d): rounding a product by a positive
        // constant is monotone
        const double cd = a.cfl * d;
        if (cd < best) best = cd;
        track_finite(nf, sp, U);
    }
    best = nonfinite_limit(best, nf);
    // wavefront minimum, then across the block's waves, then one atomic
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(best, off, 64);
        best = o < best ? o : best;
    }
    __shared__ double s_min[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_min[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = s_min[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = s_min[k] < m ? s_min[k] : m;
        fold_min(a.dt_bits, m, a.hdr);
    }
}

// octs ob..oe, or list[ob..oe) when a list is given
__global__ void k_coarse_corr(double *__restrict__ unew, const double *__restrict__ corr, int64_t corr_base,
                              const int32_t *__restrict__ nbr27, const int32_t *__restrict__ list, int64_t ob,
                              int64_t oe, int side)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = ob + t / NV;
    const int v = static_cast<int>(t % NV);
    if (i >= oe) return;
    const int64_t o = list ? int64_t(list[i]) : i;
    const int ax = side >> 1, hi = side & 1;
    const int slot = nslot(ax == 0 ? (hi ? 1 : -1) : 0, ax == 1 ? (hi ? 1 : -1) : 0, ax == 2 ? (hi ? 1 : -1) : 0);
    const int32_t e = nbr27[27 * o + slot];
    if (!(e < 0 && e != RG_NBR_OUTSIDE)) return;
    const int64_t C = -1 - int64_t(e);
    unew[NV * C + v] = unew[NV * C + v] + corr[30 * (o - corr_base) + NV * side + v];
}

// CFL limit of the coarse cells that receive coarse-fine corrections: every
// coarse face neighbour of an oct above the coarsest level
__global__ __launch_bounds__(256) void k_cfl_dt_corrected(DtArgs a, const int32_t *__restrict__ nbr27, int64_t ob,
                                                          int64_t oe)
{
    double best = __longlong_as_double(0x7ff0000000000000ll);
    double nf = 0.0;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < (oe - ob) * 6; t += stride) {
        const int64_t o = ob + t / 6;
        const int side = static_cast<int>(t % 6);
        const int ax = side >> 1, hi = side & 1;
        const int32_t e = nbr27[27 * o + nslot(ax == 0 ? (hi ? 1 : -1) : 0, ax == 1 ? (hi ? 1 : -1) : 0,
                                               ax == 2 ? (hi ? 1 : -1) : 0)];
        if (!(e < 0 && e != RG_NBR_OUTSIDE)) continue;
        const int64_t C = -1 - int64_t(e);
        int l = a.lmin;
        while (l < a.lmax && o >= a.begin[l + 1]) ++l;
        const double dx = ldexp(1.0, -(l - 1));
        double U[NV], W[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = a.u[NV * C + v];
        prim64(U, a.gamma, W);
        const double cs = sqrt_pos(div_pos(a.gamma * W[4], W[0]));
        const double sp = ((fabs(W[1]) + fabs(W[2])) + fabs(W[3])) + 3.0 * cs;
        const double cd = a.cfl * (dx / sp);
        if (cd < best) best = cd;
        track_finite(nf, sp, U);
    }
    best = nonfinite_limit(best, nf);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(best, off, 64);
        best = o < best ? o : best;
    }
    __shared__ double s_min[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_min[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = s_min[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = s_min[k] < m ? s_min[k] : m;
        fold_min(a.dt_bits, m, a.hdr);
    }
}

// children read from src, father cells written in dst (the same buffer in a
// global step; the two states of a subcycled step can differ)
__global__ void k_restrict(const double *src, double *dst, const int32_t *__restrict__ father, int64_t ob, int64_t oe)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t o = ob + t / NV;
    const int v = static_cast<int>(t % NV);
    if (o >= oe) return;
    const int32_t f = father[o];
    if (f < 0) return;   // no father cell (coarsest level): nothing to restrict into
    const double *c = src + 8 * NV * o + v;
    const double sum = ((c[0] + c[5]) + (c[10] + c[15])) + ((c[20] + c[25]) + (c[30] + c[35]));
    dst[NV * int64_t(f) + v] = 0.125 * sum;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

template <typename R, int G, int NT> rg_status launch_level(const LevelArgs &a, hipStream_t s)
{
    const int64_t n = a.oct_end - a.oct_begin;
    const unsigned blocks = static_cast<unsigned>((n + G - 1) / G);
    if (a.ghost)
        k_hydro_level<R, G, NT, true><<<blocks, NT, 0, s>>>(a);
    else
        k_hydro_level<R, G, NT, false><<<blocks, NT, 0, s>>>(a);
    return launch_status("rg_hydro_step_level");
}

template <typename R> rg_status launch_form(const LevelArgs &a, const rg_tuning *tune, hipStream_t s)
{
    const int g = tune && tune->octs_per_group ? tune->octs_per_group : 4;
    const int nt = tune && tune->threads ? tune->threads : 256;
    if (g == 4 && nt == 256) return launch_level<R, 4, 256>(a, s);
    if (g == 2 && nt == 128) return launch_level<R, 2, 128>(a, s);
    if (g == 8 && nt == 256) return launch_level<R, 8, 256>(a, s);
    if (g == 7 && nt == 256) return launch_level<R, 7, 256>(a, s);
    if (g == 3 && nt == 128) return launch_level<R, 3, 128>(a, s);
    return fail(RG_ENOTSUP, "no hydro kernel for %d octs per group and %d threads", g, nt);
}

template <typename R, int NT> rg_status launch_sib(const LevelArgs &a, const int32_t *father, hipStream_t s)
{
    const unsigned blocks = static_cast<unsigned>(a.oct_end - a.oct_begin);
    if (a.ghost)
        k_hydro_sib<R, NT, true><<<blocks, NT, 0, s>>>(a, father);
    else
        k_hydro_sib<R, NT, false><<<blocks, NT, 0, s>>>(a, father);
    return launch_status("sibling-group hydro");
}

template <typename R> rg_status launch_sib_form(const LevelArgs &a, const int32_t *father, const rg_tuning *tune,
                                                hipStream_t s)
{
    const int nt = tune && tune->group_threads ? tune->group_threads : 320;
    if (nt == 320) return launch_sib<R, 320>(a, father, s);
    if (nt == 256) return launch_sib<R, 256>(a, father, s);
    if (nt == 384) return launch_sib<R, 384>(a, father, s);
    return fail(RG_ENOTSUP, "no sibling-group kernel for %d threads", nt);
}

LevelArgs level_args(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                     const int32_t *list, int64_t count, double *corr, int64_t corr_base, const double *dt, double dx,
                     double gamma, double cfl, double *dt_next, int64_t first, const double *ucoarse, int corr_mode,
                     int ghost, const double *ucoarse2)
{
    LevelArgs a;
    a.corr_mode = corr_mode;
    a.ghost = ghost;
    a.ucoarse2 = ucoarse2 ? ucoarse2 : (ucoarse ? ucoarse : uold);
    a.list = list;
    a.uold = uold;
    a.ucoarse = ucoarse ? ucoarse : uold;
    a.unew = unew;
    a.nbr27 = nbr27;
    a.son = son;
    a.corr = corr;
    a.corr_base = corr_base;
    a.oct_begin = list ? 0 : first;
    a.oct_end = a.oct_begin + count;
    a.dt = dt;
    a.dx = dx;
    a.gamma = gamma;
    a.cfl = cfl;
    a.dt_next = reinterpret_cast<unsigned long long *>(dt_next);
    a.hdr = current_sink();
    return a;
}

}  // namespace

rg_status hydro_level(const LevelArgs &a, int form, const rg_tuning *tune, hipStream_t s)
{
    if (a.oct_end <= a.oct_begin) return RG_OK;
    if (form == RG_FP64) return launch_form<double>(a, tune, s);
    return launch_form<float>(a, tune, s);
}

// octs list[0..count) (or first..first+count when list is null)
rg_status hydro_level_list(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                           const int32_t *list, int64_t count, double *corr, int64_t corr_base, const double *dt,
                           double dx, double gamma, int form, const rg_tuning *tune, double cfl, double *dt_next,
                           hipStream_t s, int64_t first, const double *ucoarse, int corr_mode, int ghost,
                           const double *ucoarse2)
{
    if (count <= 0) return RG_OK;
    const LevelArgs a = level_args(uold, unew, nbr27, son, list, count, corr, corr_base, dt, dx, gamma, cfl, dt_next,
                                   first, ucoarse, corr_mode, ghost, ucoarse2);
    return hydro_level(a, form, tune, s);
}

// complete sibling groups whose first octs are list[0..count): octs
// list[i] .. list[i] + 7, placed in the group by their father cells
rg_status hydro_groups_list(const double *uold, double *unew, const int32_t *nbr27, const uint32_t *son,
                            const int32_t *father, const int32_t *list, int64_t count, double *corr,
                            int64_t corr_base, const double *dt, double dx, double gamma, int form,
                            const rg_tuning *tune, double cfl, double *dt_next, hipStream_t s, const double *ucoarse,
                            int corr_mode, int ghost, const double *ucoarse2)
{
    if (count <= 0) return RG_OK;
    const LevelArgs a = level_args(uold, unew, nbr27, son, list, count, corr, corr_base, dt, dx, gamma, cfl, dt_next,
                                   0, ucoarse, corr_mode, ghost, ucoarse2);
    if (form == RG_FP64) return launch_sib_form<double>(a, father, tune, s);
    return launch_sib_form<float>(a, father, tune, s);
}

// coarse-fine corrections from the octs list[0..count), side by side
rg_status coarse_corrections_list(double *unew, const double *corr, int64_t corr_base, const int32_t *nbr27,
                                  const int32_t *list, int64_t count, hipStream_t s)
{
    if (count <= 0) return RG_OK;
    const int64_t items = count * NV;
    for (int side = 0; side < 6; ++side) {
        k_coarse_corr<<<grid_for(items, 256), 256, 0, s>>>(unew, corr, corr_base, nbr27, list, 0, count, side);
        RG_TRY(launch_status("coarse corrections"));
    }
    return RG_OK;
}

// restriction of octs [ob, oe) from src into their father cells in dst
rg_status restrict_level2(const double *src, double *dst, const int32_t *father, int64_t ob, int64_t oe,
                          hipStream_t s)
{
    if (oe <= ob) return RG_OK;
    const int64_t items = (oe - ob) * NV;
    k_restrict<<<grid_for(items, 256), 256, 0, s>>>(src, dst, father, ob, oe);
    return launch_status("restrict");
}

// CFL pass; sub = 1 gives the coarse step of the subcycled scheme
rg_status cfl_dt_pass(const double *d_u, const uint32_t *d_son_mask, const int64_t *h_level_begin, int lmin, int lmax,
                      double gamma, double cfl, double *d_dt, int sub, void *stream)
{
    RG_REQUIRE(d_u && d_son_mask && h_level_begin && d_dt, "null pointer");
    RG_REQUIRE(lmin >= 1 && lmax >= lmin && lmax <= RG_MAX_LEVEL, "bad level range");
    RG_REQUIRE(gamma > 1 && cfl > 0, "bad gamma or cfl");
    RG_REQUIRE(aligned(d_dt, 8), "misaligned dt");
    DtArgs a;
    a.u = d_u;
    a.son = d_son_mask;
    for (int l = 0; l < RG_MAX_LEVEL + 2; ++l) a.begin[l] = h_level_begin[l];
    a.lmin = lmin;
    a.lmax = lmax;
    a.gamma = gamma;
    a.cfl = cfl;
    const int64_t n_oct = h_level_begin[lmax + 1] - h_level_begin[lmin];
    RG_REQUIRE(h_level_begin[lmin] == 0 && n_oct >= 0, "level ranges must start at 0");
    a.n_cell = 8 * n_oct;
    a.sub = sub;
    a.dt_bits = reinterpret_cast<unsigned long long *>(d_dt);
    a.hdr = current_sink();
    hipStream_t s = as_stream(stream);
    k_set_u64<<<1, 1, 0, s>>>(a.dt_bits, 0x7ff0000000000000ull);
    RG_TRY(launch_status("rg_cfl_dt init"));
    if (a.n_cell == 0) return RG_OK;
    const unsigned blocks = grid_for(a.n_cell, 256);
    k_cfl_dt<<<blocks < 2048 ? blocks : 2048, 256, 0, s>>>(a);
    return launch_status("rg_cfl_dt");
}

}  // namespace rg

using namespace rg;

extern "C" {

size_t rg_corr_workspace_bytes(int64_t n_octs) { return static_cast<size_t>(n_octs < 0 ? 0 : n_octs) * 30 * 8; }

rg_status rg_hydro_step_level(double dx, const double *d_dt, double gamma, const double *d_uold, double *d_unew,
                              const int32_t *d_nbr27, const uint32_t *d_son_mask, int64_t oct_begin, int64_t oct_end,
                              double *d_corr, int64_t corr_base, double cfl, double *d_dt_next, int form,
                              const rg_tuning *tune, void *stream)
{
    RG_REQUIRE(oct_begin >= 0 && oct_end >= oct_begin && oct_end <= (int64_t(1) << 28), "bad oct range");
    if (oct_end == oct_begin) return RG_OK;
    RG_REQUIRE(d_dt && d_uold && d_unew && d_nbr27 && d_son_mask, "null pointer");
    RG_REQUIRE(d_uold != d_unew, "uold and unew must not alias");
    RG_REQUIRE(aligned(d_uold, 8) && aligned(d_unew, 8) && aligned(d_dt, 8), "misaligned pointer");
    RG_REQUIRE(form == RG_FP64 || form == RG_MIXED, "bad form %d", form);
    RG_REQUIRE(dx > 0 && gamma > 1, "bad dx or gamma");
    RG_REQUIRE(!d_corr || corr_base <= oct_begin, "corr_base beyond the oct range");
    RG_REQUIRE(!d_dt_next || (cfl > 0 && aligned(d_dt_next, 8)), "bad cfl or misaligned dt_next");
    LevelArgs a;
    a.corr_mode = 0;
    a.ghost = RG_GHOST_INJECT;
    a.ucoarse2 = d_uold;
    a.list = nullptr;
    a.uold = d_uold;
    a.ucoarse = d_uold;
    a.unew = d_unew;
    a.nbr27 = d_nbr27;
    a.son = d_son_mask;
    a.corr = d_corr;
    a.corr_base = corr_base;
    a.oct_begin = oct_begin;
    a.oct_end = oct_end;
    a.dt = d_dt;
    a.dx = dx;
    a.gamma = gamma;
    a.cfl = cfl;
    a.dt_next = reinterpret_cast<unsigned long long *>(d_dt_next);
    a.hdr = current_sink();
    return hydro_level(a, form, tune, as_stream(stream));
}

rg_status rg_apply_coarse_corrections(double *d_unew, const double *d_corr, int64_t corr_base, const int32_t *d_nbr27,
                                      int64_t oct_begin, int64_t oct_end, void *stream)
{
    RG_REQUIRE(oct_begin >= 0 && oct_end >= oct_begin, "bad oct range");
    if (oct_end == oct_begin) return RG_OK;
    RG_REQUIRE(d_unew && d_corr && d_nbr27, "null pointer");
    RG_REQUIRE(corr_base <= oct_begin, "corr_base beyond the oct range");
    hipStream_t s = as_stream(stream);
    const int64_t items = (oct_end - oct_begin) * NV;
    for (int side = 0; side < 6; ++side) {
        k_coarse_corr<<<grid_for(items, 256), 256, 0, s>>>(d_unew, d_corr, corr_base, d_nbr27, nullptr, oct_begin,
                                                           oct_end, side);
        RG_TRY(launch_status("rg_apply_coarse_corrections"));
    }
    return RG_OK;
}

rg_status rg_restrict_level(double *d_u, const int32_t *d_father_cell, int64_t oct_begin, int64_t oct_end,
                            void *stream)
{
    RG_REQUIRE(oct_begin >= 0 && oct_end >= oct_begin, "bad oct range");
    if (oct_end == oct_begin) return RG_OK;
    RG_REQUIRE(d_u && d_father_cell, "null pointer");
    const int64_t items = (oct_end - oct_begin) * NV;
    k_restrict<<<grid_for(items, 256), 256, 0, as_stream(stream)>>>(d_u, d_u, d_father_cell, oct_begin, oct_end);
    return launch_status("rg_restrict_level");
}

rg_status rg_cfl_dt(const double *d_u, const uint32_t *d_son_mask, const int64_t *h_level_begin, int lmin, int lmax,
                    double gamma, double cfl, double *d_dt, void *stream)
{
    return cfl_dt_pass(d_u, d_son_mask, h_level_begin, lmin, lmax, gamma, cfl, d_dt, 0, stream);
}

rg_status rg_cfl_dt_corrected(const double *d_u, const int32_t *d_nbr27, const int64_t *h_level_begin, int lmin,
                              int lmax, double gamma, double cfl, double *d_dt, void *stream)
{
    RG_REQUIRE(d_u && d_nbr27 && h_level_begin && d_dt, "null pointer");
    RG_REQUIRE(lmin >= 1 && lmax >= lmin && lmax <= RG_MAX_LEVEL, "bad level range");
    RG_REQUIRE(gamma > 1 && cfl > 0, "bad gamma or cfl");
    RG_REQUIRE(aligned(d_dt, 8), "misaligned dt");
    if (lmax == lmin) return RG_OK;
    DtArgs a;
    a.u = d_u;
    a.son = nullptr;
    for (int l = 0; l < RG_MAX_LEVEL + 2; ++l) a.begin[l] = h_level_begin[l];
    a.lmin = lmin;
    a.lmax = lmax;
    a.gamma = gamma;
    a.cfl = cfl;
    a.n_cell = 0;
    a.sub = 0;
    a.dt_bits = reinterpret_cast<unsigned long long *>(d_dt);
    a.hdr = current_sink();
    const int64_t ob = h_level_begin[lmin + 1], oe = h_level_begin[lmax + 1];
    if (oe <= ob) return RG_OK;
    const unsigned blocks = grid_for((oe - ob) * 6, 256);
    k_cfl_dt_corrected<<<blocks < 2048 ? blocks : 2048, 256, 0, as_stream(stream)>>>(a, d_nbr27, ob, oe);
    return launch_status("rg_cfl_dt_corrected");
}

}  // extern "C"

// rg_mg.hip -- multigrid Poisson V-cycles on the oct tree.
//
// Paper Sec. 5: the self-gravity solver runs V-cycles over a hierarchy of
// levels built from the octs, with the 27-entry neighbour list replacing
// hash lookups inside the kernels; red-black Gauss-Seidel with the colours
// given by the parity of a cell's position inside its oct; the residual
// restricted by averaging the 8 children; the correction prolongated by
// trilinear interpolation with weights 27, 9, 3, 1 (/64) from the parent
// cell's neighbourhood.  Here the hierarchy is a tree whose levels lcoarse
// .. lfine are all complete (every cell below lfine split), periodic: the
// unigrid problem of the paper's measurements.  The equation is Lap phi = f
// with the 7-point Laplacian; every value is formed in the same order as in
// the serial reference so that the results agree bit for bit.
#include "rg_internal.hpp"

namespace rg {
namespace {

// the six face-neighbour cells of cell c of oct o, in the order x-, x+, y-,
// y+, z-, z+ (same oct, else the neighbouring oct through the list)
__device__ __forceinline__ void face_cells(const int32_t *__restrict__ nbr27, int64_t o, int c, int64_t *nb)
{
    const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
#pragma unroll
    for (int side = 0; side < 6; ++side) {
        const int ax = side >> 1, d = (side & 1) ? 1 : -1;
        int p[3] = {cx, cy, cz};
        p[ax] += d;
        if (p[ax] >= 0 && p[ax] <= 1) {
            nb[side] = 8 * o + (p[0] + 2 * p[1] + 4 * p[2]);
        } else {
            const int slot = 13 + (ax == 0 ? d : ax == 1 ? 3 * d : 9 * d);
            const int32_t e = nbr27[27 * o + slot];
            nb[side] = 8 * int64_t(e) + ((p[0] & 1) + 2 * (p[1] & 1) + 4 * (p[2] & 1));
        }
    }
}

__device__ __forceinline__ double sum6(const double *__restrict__ phi, const int64_t *nb)
{
    return ((((phi[nb[0]] + phi[nb[1]]) + phi[nb[2]]) + phi[nb[3]]) + phi[nb[4]]) + phi[nb[5]];
}

// cells of one colour: even (0, 3, 5, 6) or odd (1, 2, 4, 7) coordinate sum
__constant__ int c_colour[2][4] = {{0, 3, 5, 6}, {1, 2, 4, 7}};

// Gauss-Seidel update of cell c of oct o
__device__ __forceinline__ void smooth_cell(double *phi, const double *f, const int32_t *__restrict__ nbr27, int64_t o,
                                            int c, double h2)
{
    int64_t nb[6];
    face_cells(nbr27, o, c, nb);
    const int64_t cell = 8 * o + c;
    phi[cell] = (sum6(phi, nb) - h2 * f[cell]) / 6.0;
}

__device__ __forceinline__ void residual_cell(const double *phi, const double *f, double *r,
                                              const int32_t *__restrict__ nbr27, int64_t o, int c, double h2)
{
    int64_t nb[6];
    face_cells(nbr27, o, c, nb);
    const int64_t cell = 8 * o + c;
    const double lap = (sum6(phi, nb) - 6.0 * phi[cell]) / h2;
    r[cell] = f[cell] - lap;
}

// coarse right-hand side at fine oct o's father cell: the mean of the 8
// fine residuals, summed pairwise in cell order
__device__ __forceinline__ void restrict_oct(const double *r, double *f, const int32_t *__restrict__ father, int64_t o)
{
    const double *c = r + 8 * o;
    f[father[o]] = 0.125 * (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7])));
}

// one colour pass of Gauss-Seidel over the octs [ob, oe): four cells per oct
__global__ void k_mg_smooth(double *phi, const double *__restrict__ f, const int32_t *__restrict__ nbr27, int64_t ob,
                            int64_t oe, double h2, int colour)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t o = ob + (t >> 2);
    if (o >= oe) return;
    smooth_cell(phi, f, nbr27, o, c_colour[colour][t & 3], h2);
}

__global__ void k_mg_residual(const double *__restrict__ phi, const double *__restrict__ f, double *__restrict__ r,
                              const int32_t *__restrict__ nbr27, int64_t ob, int64_t oe, double h2)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t o = ob + (t >> 3);
    if (o >= oe) return;
    residual_cell(phi, f, r, nbr27, o, static_cast<int>(t & 7), h2);
}

__global__ void k_mg_restrict(const double *__restrict__ r, double *__restrict__ f, const int32_t *__restrict__ father,
                              int64_t ob, int64_t oe)
{
    const int64_t o = ob + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= oe) return;
    restrict_oct(r, f, father, o);
}

__global__ void k_mg_zero(double *p, int64_t b, int64_t e)
{
    const int64_t i = b + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < e) p[i] = 0.0;
}

// phi of each fine cell += trilinear interpolation of the coarse correction:
// the fine cell sits a quarter of its father cell C's width from C's centre
// toward side s per axis; the 8 coarse cells C + {0, s_x} x {0, s_y} x {0,
// s_z} weigh 27, 9, 3, 1 by the number of steps
__device__ __forceinline__ void prolong_cell(double *phi, const int32_t *__restrict__ nbr27,
                                             const int32_t *__restrict__ father, int64_t o, int c)
{
    const int64_t C = father[o];
    const int64_t P = C >> 3;
    const int q = static_cast<int>(C & 7);
    const int q3[3] = {q & 1, (q >> 1) & 1, q >> 2};
    const int s3[3] = {(c & 1) ? 1 : -1, ((c >> 1) & 1) ? 1 : -1, (c >> 2) ? 1 : -1};
    double e[8];   // index b: bit a set = one step along axis a
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        int p[3], sl[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a] = q3[a] + (((b >> a) & 1) ? s3[a] : 0);
            sl[a] = p[a] < 0 ? -1 : (p[a] > 1 ? 1 : 0);
        }
        int64_t cell;
        if (sl[0] == 0 && sl[1] == 0 && sl[2] == 0) {
            cell = 8 * P + (p[0] + 2 * p[1] + 4 * p[2]);
        } else {
            const int32_t n = nbr27[27 * P + (sl[0] + 1) + 3 * (sl[1] + 1) + 9 * (sl[2] + 1)];
            cell = 8 * int64_t(n) + ((p[0] & 1) + 2 * (p[1] & 1) + 4 * (p[2] & 1));
        }
        e[b] = phi[cell];
    }
    const double w = ((((((27.0 * e[0] + 9.0 * e[1]) + 9.0 * e[2]) + 9.0 * e[4]) + 3.0 * e[3]) + 3.0 * e[5]) +
                      3.0 * e[6]) + e[7];
    const int64_t cell = 8 * o + c;
    phi[cell] = phi[cell] + 0.015625 * w;
}

__global__ void k_mg_prolong(double *phi, const int32_t *__restrict__ nbr27, const int32_t *__restrict__ father,
                             int64_t ob, int64_t oe)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t o = ob + (t >> 3);
    if (o >= oe) return;
    prolong_cell(phi, nbr27, father, o, static_cast<int>(t & 7));
}

// The levels of at most kTailOcts octs (those below lfine's first such
// level are smaller still) run their whole part of the V-cycle in one
// workgroup: the same passes in the same order as the per-level launches,
// separated by barriers, so the same bits.  Each launch (two per sweep, 100
// for 50 sweeps on the coarsest level) costs a few microseconds of GPU time.
constexpr int64_t kTailOcts = 512;
constexpr int kTailThreads = 1024;

struct MgTail {
    double *phi, *f, *r;
    const int32_t *nbr27, *father;
    int64_t begin[RG_MAX_LEVEL + 2];
    double h2[RG_MAX_LEVEL + 1];
    int m0, lcoarse, nu1, nu2, ncoarse;
};

__device__ void tail_sweeps(const MgTail &A, int l, int sweeps)
{
    const int64_t ob = A.begin[l], n4 = 4 * (A.begin[l + 1] - ob);
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t t = threadIdx.x; t < n4; t += blockDim.x)
                smooth_cell(A.phi, A.f, A.nbr27, ob + (t >> 2), c_colour[colour][t & 3], A.h2[l]);
            __syncthreads();
        }
}

// The coarsest level's sweeps (50 by default, each pass depending on the
// last) with its values staged in LDS when it holds at most kLdsCells cells:
// the same update of each cell, read from and written to LDS.
constexpr int kLdsCells = 1024;

__device__ void tail_sweeps_lds(const MgTail &A, int l, int sweeps, double *sp, double *sf)
{
    const int64_t ob = A.begin[l], cb = 8 * ob, n = 8 * (A.begin[l + 1] - ob);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        sp[i] = A.phi[cb + i];
        sf[i] = A.f[cb + i];
    }
    __syncthreads();
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t t = threadIdx.x; t < n / 2; t += blockDim.x) {
                const int64_t o = ob + (t >> 2);
                const int c = c_colour[colour][t & 3];
                int64_t nb[6];
                face_cells(A.nbr27, o, c, nb);
                const double s6 = ((((sp[nb[0] - cb] + sp[nb[1] - cb]) + sp[nb[2] - cb]) + sp[nb[3] - cb]) +
                                   sp[nb[4] - cb]) + sp[nb[5] - cb];
                const int64_t k = 8 * o + c - cb;
                sp[k] = (s6 - A.h2[l] * sf[k]) / 6.0;
            }
            __syncthreads();
        }
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) A.phi[cb + i] = sp[i];
    __syncthreads();
}

__global__ __launch_bounds__(kTailThreads) void k_mg_tail(MgTail A)
{
    __shared__ double sp[kLdsCells], sf[kLdsCells];
    for (int l = A.m0; l > A.lcoarse; --l) {
        tail_sweeps(A, l, A.nu1);
        const int64_t ob = A.begin[l], oe = A.begin[l + 1];
        for (int64_t t = threadIdx.x; t < 8 * (oe - ob); t += blockDim.x)
            residual_cell(A.phi, A.f, A.r, A.nbr27, ob + (t >> 3), static_cast<int>(t & 7), A.h2[l]);
        __syncthreads();
        for (int64_t o = ob + threadIdx.x; o < oe; o += blockDim.x) restrict_oct(A.r, A.f, A.father, o);
        for (int64_t i = 8 * A.begin[l - 1] + threadIdx.x; i < 8 * A.begin[l]; i += blockDim.x) A.phi[i] = 0.0;
        __syncthreads();
    }
    if (8 * (A.begin[A.lcoarse + 1] - A.begin[A.lcoarse]) <= kLdsCells)
        tail_sweeps_lds(A, A.lcoarse, A.ncoarse, sp, sf);
    else
        tail_sweeps(A, A.lcoarse, A.ncoarse);
    for (int l = A.lcoarse + 1; l <= A.m0; ++l) {
        const int64_t ob = A.begin[l], oe = A.begin[l + 1];
        for (int64_t t = threadIdx.x; t < 8 * (oe - ob); t += blockDim.x)
            prolong_cell(A.phi, A.nbr27, A.father, ob + (t >> 3), static_cast<int>(t & 7));
        __syncthreads();
        tail_sweeps(A, l, A.nu2);
    }
}

struct Mg {
    const rg_tree *t;
    double *phi, *f, *r;
    int lcoarse, nu1, nu2, ncoarse;
    hipStream_t s;
};

rg_status smooth(const Mg &m, int l, int sweeps)
{
    const int64_t ob = m.t->level_begin[l], oe = m.t->level_begin[l + 1];
    const double h2 = ldexp(1.0, -2 * l);
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            k_mg_smooth<<<grid_for(4 * (oe - ob), 256), 256, 0, m.s>>>(m.phi, m.f, m.t->d_nbr27, ob, oe, h2, colour);
            RG_TRY(launch_status("multigrid smooth"));
        }
    return RG_OK;
}

rg_status residual(const rg_tree *t, const double *phi, const double *f, double *r, int l, hipStream_t s)
{
    const int64_t ob = t->level_begin[l], oe = t->level_begin[l + 1];
    k_mg_residual<<<grid_for(8 * (oe - ob), 256), 256, 0, s>>>(phi, f, r, t->d_nbr27, ob, oe, ldexp(1.0, -2 * l));
    return launch_status("multigrid residual");
}

rg_status vcycle(const Mg &m, int l)
{
    const rg_tree *t = m.t;
    if (t->level_begin[l + 1] - t->level_begin[l] <= kTailOcts) {
        MgTail A;
        A.phi = m.phi;
        A.f = m.f;
        A.r = m.r;
        A.nbr27 = t->d_nbr27;
        A.father = t->d_father_cell;
        for (int k = 0; k <= RG_MAX_LEVEL + 1; ++k) A.begin[k] = t->level_begin[k];
        for (int k = 0; k <= RG_MAX_LEVEL; ++k) A.h2[k] = ldexp(1.0, -2 * k);
        A.m0 = l;
        A.lcoarse = m.lcoarse;
        A.nu1 = m.nu1;
        A.nu2 = m.nu2;
        A.ncoarse = m.ncoarse;
        k_mg_tail<<<1, kTailThreads, 0, m.s>>>(A);
        return launch_status("multigrid small levels");
    }
    if (l == m.lcoarse) return smooth(m, l, m.ncoarse);
    RG_TRY(smooth(m, l, m.nu1));
    RG_TRY(residual(t, m.phi, m.f, m.r, l, m.s));
    const int64_t ob = t->level_begin[l], oe = t->level_begin[l + 1];
    k_mg_restrict<<<grid_for(oe - ob, 256), 256, 0, m.s>>>(m.r, m.f, t->d_father_cell, ob, oe);
    RG_TRY(launch_status("multigrid restrict"));
    const int64_t cb = 8 * t->level_begin[l - 1], ce = 8 * t->level_begin[l];
    k_mg_zero<<<grid_for(ce - cb, 256), 256, 0, m.s>>>(m.phi, cb, ce);
    RG_TRY(launch_status("multigrid zero"));
    RG_TRY(vcycle(m, l - 1));
    k_mg_prolong<<<grid_for(8 * (oe - ob), 256), 256, 0, m.s>>>(m.phi, t->d_nbr27, t->d_father_cell, ob, oe);
    RG_TRY(launch_status("multigrid prolong"));
    return smooth(m, l, m.nu2);
}

rg_status check_hierarchy(const rg_tree *t, int lfine, int lcoarse)
{
    RG_REQUIRE(t && t->d_nbr27 && t->d_father_cell, "tree without neighbour lists");
    RG_REQUIRE(t->bc == RG_BC_PERIODIC, "the multigrid hierarchy must be periodic");
    RG_REQUIRE(lcoarse >= 1 && lcoarse <= lfine && lfine <= t->lmax && lcoarse >= t->lmin && lfine <= 10,
               "levels %d..%d not in the tree", lcoarse, lfine);
    for (int l = lcoarse; l <= lfine; ++l)
        RG_REQUIRE(t->level_begin[l + 1] - t->level_begin[l] == (int64_t(1) << (3 * (l - 1))),
                   "level %d is not complete", l);
    return RG_OK;
}

}  // namespace
}  // namespace rg

using namespace rg;

extern "C" {

rg_status rg_mg_residual(const rg_tree *t, const double *d_phi, const double *d_f, double *d_r, int level,
                         void *stream)
{
    RG_TRY(check_hierarchy(t, level, level));
    RG_REQUIRE(d_phi && d_f && d_r, "null pointer");
    return residual(t, d_phi, d_f, d_r, level, as_stream(stream));
}

rg_status rg_mg_vcycles(const rg_tree *t, double *d_phi, double *d_f, double *d_r, int lfine, int lcoarse, int nu1,
                        int nu2, int ncoarse, int ncycles, void *stream)
{
    RG_TRY(check_hierarchy(t, lfine, lcoarse));
    RG_REQUIRE(d_phi && d_f && d_r, "null pointer");
    RG_REQUIRE(nu1 >= 0 && nu2 >= 0 && ncoarse >= 0 && ncycles >= 0, "negative sweep or cycle count");
    Mg m;
    m.t = t;
    m.phi = d_phi;
    m.f = d_f;
    m.r = d_r;
    m.lcoarse = lcoarse;
    m.nu1 = nu1;
    m.nu2 = nu2;
    m.ncoarse = ncoarse;
    m.s = as_stream(stream);
    for (int c = 0; c < ncycles; ++c) RG_TRY(vcycle(m, lfine));
    return RG_OK;
}

}  // extern "C"

// rg_mg_amr.hip -- multigrid Poisson V-cycles on one level of an AMR tree.
//
// Paper Sec. 5: the potential is built level by level with V-cycles;
// red-black Gauss-Seidel with the colours given by the parity of a cell's
// position inside its oct, its diagonal adjusted in cells that the level's
// boundary cuts (located by a signed-distance-like mask); residuals
// restricted by the mean of the 8 children; corrections prolongated by
// trilinear interpolation with weights 27, 9, 3, 1 (/64) from the parent
// cell's neighbourhood; neighbours through a 27-entry list built once from
// hash lookups.
//
// Level L's unknowns are the potential of the cells of its octs.  A face
// neighbour outside the level lies in a leaf of level L-1 (the tree is
// graded): its value is the trilinear interpolation of level L-1's
// potential at its centre, fixed while level L is solved.  The coarse
// levels of the V-cycle hold the ancestors of level L's octs down to
// lcoarse (keys K >> 3, deduplicated level by level), in one oct array with
// its own hash table and same-level neighbour lists (-1 where no such oct
// exists).  mask = +1 on level L's cells; on a coarse cell the mean of its
// children's masks, -1 without children.  A coarse cell is inside when its
// mask is positive; an outside neighbour j of inside cell i puts e = 0 at
// the fraction m_i / (m_i - m_j) of the way and adds (m_i - m_j) / m_i - 1
// to the Gauss-Seidel diagonal.  Every value is formed in the same order as
// in the serial reference so that the results agree bit for bit.
#include "rg_internal.hpp"

#include <hipcub/hipcub.hpp>

#include <vector>

struct rg_mg_level {
    int level, lcoarse;
    int64_t fine_begin, n_fine;          // the level's octs in the tree
    int64_t tree_n_oct;
    int64_t mg_begin[RG_MAX_LEVEL + 2];  // coarse octs of level m: [mg_begin[m], mg_begin[m + 1])
    int64_t n_mg;
    void *mem;
    uint64_t *keys;                      // [n_mg] coarse keys, level by level, key order
    int32_t *nbr;                        // [n_mg][27] same-level coarse oct, -1 if none
    int32_t *father;                     // [n_mg] coarse cell of the father, -1 on lcoarse
    int32_t *fine_father;                // [n_fine] coarse cell of each fine oct's father
    double *e, *f, *r, *mask;            // [8 n_mg]
    double *rfine;                       // [8 n_fine]
    void *hash_ws;
};

namespace rg {
namespace {

__device__ __forceinline__ int cell_of(const int p[3]) { return (p[0] & 1) + 2 * (p[1] & 1) + 4 * (p[2] & 1); }

// value of face neighbour `side` (x-, x+, y-, y+, z-, z+) of fine cell c of
// tree oct o: a level-L cell, or the interpolated level-(L-1) potential
__device__ __forceinline__ double fine_neighbour(const double *phi, const int32_t *__restrict__ nbr27,
                                                 const int32_t *__restrict__ fcell, int64_t o, int c, int side)
{
    const int ax = side >> 1, d = (side & 1) ? 1 : -1;
    int p[3] = {c & 1, (c >> 1) & 1, c >> 2};
    p[ax] += d;
    if (p[ax] >= 0 && p[ax] <= 1) return phi[8 * o + cell_of(p)];
    int dv[3] = {0, 0, 0};
    dv[ax] = d;
    const int32_t e = nbr27[27 * o + 13 + dv[0] + 3 * dv[1] + 9 * dv[2]];
    if (e >= 0) return phi[8 * int64_t(e) + cell_of(p)];
    // the neighbour sits in coarse cell F + dv (F the father of o), toward
    // side s of that cell's centre; the 8 coarse cells F + dv + {0, s}^3
    int s[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = (p[a] & 1) ? 1 : -1;
    double v[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        int D[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) D[a] = dv[a] + (((b >> a) & 1) ? s[a] : 0);
        const int32_t n = nbr27[27 * o + 13 + D[0] + 3 * D[1] + 9 * D[2]];
        const int64_t cell = n >= 0 ? int64_t(fcell[n]) : int64_t(-1 - n);
        v[b] = phi[cell];
    }
    const double w = ((((((27.0 * v[0] + 9.0 * v[1]) + 9.0 * v[2]) + 9.0 * v[4]) + 3.0 * v[3]) + 3.0 * v[5]) +
                      3.0 * v[6]) + v[7];
    return 0.015625 * w;
}

__device__ __forceinline__ double fine_sum6(const double *phi, const int32_t *__restrict__ nbr27,
                                            const int32_t *__restrict__ fcell, int64_t o, int c)
{
    return ((((fine_neighbour(phi, nbr27, fcell, o, c, 0) + fine_neighbour(phi, nbr27, fcell, o, c, 1)) +
              fine_neighbour(phi, nbr27, fcell, o, c, 2)) + fine_neighbour(phi, nbr27, fcell, o, c, 3)) +
            fine_neighbour(phi, nbr27, fcell, o, c, 4)) + fine_neighbour(phi, nbr27, fcell, o, c, 5);
}

__constant__ int c_amr_colour[2][4] = {{0, 3, 5, 6}, {1, 2, 4, 7}};

__global__ void k_fine_smooth(double *phi, const double *__restrict__ f, const int32_t *__restrict__ nbr27,
                              const int32_t *__restrict__ fcell, int64_t ob, int64_t oe, double h2, int colour)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t o = ob + (t >> 2);
    if (o >= oe) return;
    const int c = c_amr_colour[colour][t & 3];
    const int64_t cell = 8 * o + c;
    phi[cell] = (fine_sum6(phi, nbr27, fcell, o, c) - h2 * f[cell]) / 6.0;
}

// r of every fine cell, at out[8 (o - out_base) + c]
__global__ void k_fine_residual(const double *__restrict__ phi, const double *__restrict__ f,
                                const int32_t *__restrict__ nbr27, const int32_t *__restrict__ fcell, int64_t ob,
                                int64_t oe, double h2, double *__restrict__ out, int64_t out_base)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t o = ob + (t >> 3);
    if (o >= oe) return;
    const int c = static_cast<int>(t & 7);
    const int64_t cell = 8 * o + c;
    const double lap = (fine_sum6(phi, nbr27, fcell, o, c) - 6.0 * phi[cell]) / h2;
    out[8 * (o - out_base) + c] = f[cell] - lap;
}

// inside-neighbour sum s and diagonal excess d of coarse cell c of oct g
__device__ __forceinline__ void coarse_terms(const double *e, const double *__restrict__ mask,
                                             const int32_t *__restrict__ nbr, int64_t g, int c, double mi, double &s,
                                             double &d)
{
    s = 0.0;
    d = 0.0;
#pragma unroll
    for (int side = 0; side < 6; ++side) {
        const int ax = side >> 1, dd = (side & 1) ? 1 : -1;
        int p[3] = {c & 1, (c >> 1) & 1, c >> 2};
        p[ax] += dd;
        int64_t j = -1;
        if (p[ax] >= 0 && p[ax] <= 1) {
            j = 8 * g + cell_of(p);
        } else {
            const int32_t n = nbr[27 * g + 13 + (ax == 0 ? dd : ax == 1 ? 3 * dd : 9 * dd)];
            if (n >= 0) j = 8 * int64_t(n) + cell_of(p);
        }
        const double mj = j >= 0 ? mask[j] : -1.0;
        if (mj > 0.0)
            s = s + e[j];
        else
            d = d + ((mi - mj) / mi - 1.0);
    }
}

__global__ void k_coarse_smooth(double *e, const double *__restrict__ f, const double *__restrict__ mask,
                                const int32_t *__restrict__ nbr, int64_t gb, int64_t ge, double h2, int colour)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t g = gb + (t >> 2);
    if (g >= ge) return;
    const int c = c_amr_colour[colour][t & 3];
    const int64_t cell = 8 * g + c;
    const double mi = mask[cell];
    if (!(mi > 0.0)) return;
    double s, d;
    coarse_terms(e, mask, nbr, g, c, mi, s, d);
    e[cell] = (s - h2 * f[cell]) / (6.0 + d);
}

__global__ void k_coarse_residual(const double *__restrict__ e, const double *__restrict__ f,
                                  const double *__restrict__ mask, const int32_t *__restrict__ nbr, int64_t gb,
                                  int64_t ge, double h2, double *__restrict__ r)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t g = gb + (t >> 3);
    if (g >= ge) return;
    const int c = static_cast<int>(t & 7);
    const int64_t cell = 8 * g + c;
    const double mi = mask[cell];
    if (!(mi > 0.0)) {
        r[cell] = 0.0;
        return;
    }
    double s, d;
    coarse_terms(e, mask, nbr, g, c, mi, s, d);
    const double lap = (s - (6.0 + d) * e[cell]) / h2;
    r[cell] = f[cell] - lap;
}

// dst[father[o]] = mean of src[8 o .. 8 o + 7], summed pairwise in cell order
// (src and dst may be one array: the children and the fathers are on
// different levels)
__global__ void k_restrict8(const double *src, const int32_t *__restrict__ father, int64_t ob, int64_t oe, double *dst)
{
    const int64_t o = ob + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= oe) return;
    const double *c = src + 8 * o;
    dst[father[o]] = 0.125 * (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7])));
}

__global__ void k_fill(double *p, int64_t b, int64_t e, double v)
{
    const int64_t i = b + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < e) p[i] = v;
}

__global__ void k_mask_level_above_fine(const int32_t *__restrict__ fine_father, int64_t n, double *mask)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o < n) mask[fine_father[o]] = 1.0;   // the mean of eight +1
}

// the correction of the coarse cells around cell c's father cell C,
// interpolated at c (absent coarse cells hold 0)
__device__ __forceinline__ double prolong_value(const double *e, const int32_t *__restrict__ nbr,
                                                int32_t C, int c)
{
    const int64_t P = C >> 3;
    const int q = C & 7;
    const int q3[3] = {q & 1, (q >> 1) & 1, q >> 2};
    const int s3[3] = {(c & 1) ? 1 : -1, ((c >> 1) & 1) ? 1 : -1, (c >> 2) ? 1 : -1};
    double v[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        int p[3], sl[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a] = q3[a] + (((b >> a) & 1) ? s3[a] : 0);
            sl[a] = p[a] < 0 ? -1 : (p[a] > 1 ? 1 : 0);
        }
        if (sl[0] == 0 && sl[1] == 0 && sl[2] == 0) {
            v[b] = e[8 * P + cell_of(p)];
        } else {
            const int32_t n = nbr[27 * P + (sl[0] + 1) + 3 * (sl[1] + 1) + 9 * (sl[2] + 1)];
            v[b] = n >= 0 ? e[8 * int64_t(n) + cell_of(p)] : 0.0;
        }
    }
    const double w = ((((((27.0 * v[0] + 9.0 * v[1]) + 9.0 * v[2]) + 9.0 * v[4]) + 3.0 * v[3]) + 3.0 * v[5]) +
                      3.0 * v[6]) + v[7];
    return 0.015625 * w;
}

__global__ void k_prolong_fine(double *phi, const double *__restrict__ e, const int32_t *__restrict__ nbr,
                               const int32_t *__restrict__ fine_father, int64_t ob, int64_t n_fine)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t ol = t >> 3;
    if (ol >= n_fine) return;
    const int c = static_cast<int>(t & 7);
    const int64_t cell = 8 * (ob + ol) + c;
    phi[cell] = phi[cell] + prolong_value(e, nbr, fine_father[ol], c);
}

__global__ void k_prolong_coarse(double *e, const double *__restrict__ mask, const int32_t *__restrict__ nbr,
                                 const int32_t *__restrict__ father, int64_t gb, int64_t ge)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t g = gb + (t >> 3);
    if (g >= ge) return;
    const int c = static_cast<int>(t & 7);
    const int64_t cell = 8 * g + c;
    if (!(mask[cell] > 0.0)) return;
    e[cell] = e[cell] + prolong_value(e, nbr, father[g], c);
}

// ---------------------------------------------------------------- small levels
//
// The coarse levels with at most kTailOcts octs (all levels below the first
// such level are smaller still) run their whole part of the V-cycle in one
// workgroup: the same passes in the same order as the per-level launches,
// separated by barriers instead of kernel boundaries, so the results are the
// same bits.  Each of those launches (two per sweep, 100 for 50 sweeps on
// the coarsest level) costs a few microseconds of GPU time however little
// it does.

constexpr int64_t kTailOcts = 512;
constexpr int kTailThreads = 1024;

struct TailArgs {
    double *e, *f, *r;
    const double *mask;
    const int32_t *nbr, *father;
    int64_t begin[RG_MAX_LEVEL + 2];
    double h2[RG_MAX_LEVEL + 1];
    int m0, lcoarse, nu1, nu2, ncoarse;
};

__device__ void tail_smooth(const TailArgs &A, int m, int sweeps)
{
    const int64_t gb = A.begin[m], n4 = 4 * (A.begin[m + 1] - gb);
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t t = threadIdx.x; t < n4; t += blockDim.x) {
                const int64_t g = gb + (t >> 2);
                const int c = c_amr_colour[colour][t & 3];
                const int64_t cell = 8 * g + c;
                const double mi = A.mask[cell];
                if (!(mi > 0.0)) continue;
                double s, d;
                coarse_terms(A.e, A.mask, A.nbr, g, c, mi, s, d);
                A.e[cell] = (s - A.h2[m] * A.f[cell]) / (6.0 + d);
            }
            __syncthreads();
        }
}

// The coarsest level's sweeps (50 by default, each pass depending on the
// last) with its corrections, right-hand sides and masks staged in LDS when
// it holds at most kLdsCells cells: the same update of each cell.
constexpr int kLdsCells = 1024;

__device__ void tail_sweeps_lds(const TailArgs &A, int m, int sweeps, double *se, double *sf, double *sm)
{
    const int64_t gb = A.begin[m], cb = 8 * gb, n = 8 * (A.begin[m + 1] - gb);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        se[i] = A.e[cb + i];
        sf[i] = A.f[cb + i];
        sm[i] = A.mask[cb + i];
    }
    __syncthreads();
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            for (int64_t t = threadIdx.x; t < n / 2; t += blockDim.x) {
                const int64_t g = gb + (t >> 2);
                const int c = c_amr_colour[colour][t & 3];
                const int64_t k = 8 * g + c - cb;
                const double mi = sm[k];
                if (!(mi > 0.0)) continue;
                double s = 0.0, d = 0.0;
#pragma unroll
                for (int side = 0; side < 6; ++side) {
                    const int ax = side >> 1, dd = (side & 1) ? 1 : -1;
                    int p[3] = {c & 1, (c >> 1) & 1, c >> 2};
                    p[ax] += dd;
                    int64_t j = -1;
                    if (p[ax] >= 0 && p[ax] <= 1) {
                        j = 8 * g + cell_of(p);
                    } else {
                        const int32_t nn = A.nbr[27 * g + 13 + (ax == 0 ? dd : ax == 1 ? 3 * dd : 9 * dd)];
                        if (nn >= 0) j = 8 * int64_t(nn) + cell_of(p);
                    }
                    const double mj = j >= 0 ? sm[j - cb] : -1.0;
                    if (mj > 0.0)
                        s = s + se[j - cb];
                    else
                        d = d + ((mi - mj) / mi - 1.0);
                }
                se[k] = (s - A.h2[m] * sf[k]) / (6.0 + d);
            }
            __syncthreads();
        }
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) A.e[cb + i] = se[i];
    __syncthreads();
}

__global__ __launch_bounds__(kTailThreads) void k_vcycle_tail(TailArgs A)
{
    __shared__ double se[kLdsCells], sf[kLdsCells], sm[kLdsCells];
    for (int m = A.m0; m > A.lcoarse; --m) {
        tail_smooth(A, m, A.nu1);
        const int64_t gb = A.begin[m], ge = A.begin[m + 1];
        for (int64_t t = threadIdx.x; t < 8 * (ge - gb); t += blockDim.x) {
            const int64_t g = gb + (t >> 3);
            const int c = static_cast<int>(t & 7);
            const int64_t cell = 8 * g + c;
            const double mi = A.mask[cell];
            if (!(mi > 0.0)) {
                A.r[cell] = 0.0;
                continue;
            }
            double s, d;
            coarse_terms(A.e, A.mask, A.nbr, g, c, mi, s, d);
            const double lap = (s - (6.0 + d) * A.e[cell]) / A.h2[m];
            A.r[cell] = A.f[cell] - lap;
        }
        for (int64_t i = 8 * A.begin[m - 1] + threadIdx.x; i < 8 * A.begin[m]; i += blockDim.x) {
            A.f[i] = 0.0;
            A.e[i] = 0.0;
        }
        __syncthreads();
        for (int64_t g = gb + threadIdx.x; g < ge; g += blockDim.x) {
            const double *c = A.r + 8 * g;
            A.f[A.father[g]] = 0.125 * (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7])));
        }
        __syncthreads();
    }
    if (8 * (A.begin[A.lcoarse + 1] - A.begin[A.lcoarse]) <= kLdsCells)
        tail_sweeps_lds(A, A.lcoarse, A.ncoarse, se, sf, sm);
    else
        tail_smooth(A, A.lcoarse, A.ncoarse);
    for (int m = A.lcoarse + 1; m <= A.m0; ++m) {
        const int64_t gb = A.begin[m], ge = A.begin[m + 1];
        for (int64_t t = threadIdx.x; t < 8 * (ge - gb); t += blockDim.x) {
            const int64_t g = gb + (t >> 3);
            const int c = static_cast<int>(t & 7);
            const int64_t cell = 8 * g + c;
            if (!(A.mask[cell] > 0.0)) continue;
            A.e[cell] = A.e[cell] + prolong_value(A.e, A.nbr, A.father[g], c);
        }
        __syncthreads();
        tail_smooth(A, m, A.nu2);
    }
}

// ---------------------------------------------------------------- build

__global__ void k_shift3(const uint64_t *__restrict__ in, int64_t n, uint64_t *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] >> 3;
}

__global__ void k_coarse_links(const uint64_t *__restrict__ keys, int64_t n, HashView h, int lcoarse,
                               int32_t *__restrict__ nbr, int32_t *__restrict__ father)
{
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    int32_t i, j, k, l;
    key_coords(keys[g], i, j, k, l);
    const int32_t side = int32_t(1) << (l - 1);
    for (int d = 0; d < 27; ++d) {
        const int32_t ii = (i + (d % 3) - 1 + side) % side, jj = (j + (d / 3) % 3 - 1 + side) % side,
                      kk = (k + d / 9 - 1 + side) % side;
        nbr[27 * g + d] = hash_probe(h.keys, h.vals, h.mask, oct_key(ii, jj, kk, l));
    }
    father[g] = l > lcoarse ? 8 * hash_probe(h.keys, h.vals, h.mask, keys[g] >> 3) + ((i & 1) + 2 * (j & 1) + 4 * (k & 1))
                            : -1;
}

__global__ void k_fine_links(const uint64_t *__restrict__ keys, int64_t n, HashView h, int32_t *__restrict__ fine_father)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    int32_t i, j, k, l;
    key_coords(keys[o], i, j, k, l);
    fine_father[o] = 8 * hash_probe(h.keys, h.vals, h.mask, keys[o] >> 3) + ((i & 1) + 2 * (j & 1) + 4 * (k & 1));
}

inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

struct Ctx {
    const rg_tree *t;
    rg_mg_level *h;
    double *phi;
    const double *f;
    int nu1, nu2, ncoarse;
    hipStream_t s;
};

rg_status fine_smooth(const Ctx &x, int sweeps)
{
    const rg_mg_level *h = x.h;
    const int64_t ob = h->fine_begin, oe = ob + h->n_fine;
    const double h2 = ldexp(1.0, -2 * h->level);
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            k_fine_smooth<<<grid_for(4 * h->n_fine, 256), 256, 0, x.s>>>(x.phi, x.f, x.t->d_nbr27, x.t->d_father_cell,
                                                                        ob, oe, h2, colour);
            RG_TRY(launch_status("level multigrid smooth"));
        }
    return RG_OK;
}

rg_status coarse_smooth(const Ctx &x, int m, int sweeps)
{
    const rg_mg_level *h = x.h;
    const int64_t gb = h->mg_begin[m], ge = h->mg_begin[m + 1];
    const double h2 = ldexp(1.0, -2 * m);
    for (int sw = 0; sw < sweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour) {
            k_coarse_smooth<<<grid_for(4 * (ge - gb), 256), 256, 0, x.s>>>(h->e, h->f, h->mask, h->nbr, gb, ge, h2,
                                                                          colour);
            RG_TRY(launch_status("level multigrid coarse smooth"));
        }
    return RG_OK;
}

rg_status fill(double *p, int64_t b, int64_t e, double v, hipStream_t s)
{
    if (e <= b) return RG_OK;
    k_fill<<<grid_for(e - b, 256), 256, 0, s>>>(p, b, e, v);
    return launch_status("level multigrid fill");
}

rg_status vcoarse(const Ctx &x, int m)
{
    rg_mg_level *h = x.h;
    if (h->mg_begin[m + 1] - h->mg_begin[m] <= kTailOcts) {
        TailArgs A;
        A.e = h->e;
        A.f = h->f;
        A.r = h->r;
        A.mask = h->mask;
        A.nbr = h->nbr;
        A.father = h->father;
        for (int k = 0; k <= RG_MAX_LEVEL + 1; ++k) A.begin[k] = h->mg_begin[k];
        for (int k = 0; k <= RG_MAX_LEVEL; ++k) A.h2[k] = ldexp(1.0, -2 * k);
        A.m0 = m;
        A.lcoarse = h->lcoarse;
        A.nu1 = x.nu1;
        A.nu2 = x.nu2;
        A.ncoarse = x.ncoarse;
        k_vcycle_tail<<<1, kTailThreads, 0, x.s>>>(A);
        return launch_status("level multigrid small levels");
    }
    if (m == h->lcoarse) return coarse_smooth(x, m, x.ncoarse);
    RG_TRY(coarse_smooth(x, m, x.nu1));
    const int64_t gb = h->mg_begin[m], ge = h->mg_begin[m + 1];
    k_coarse_residual<<<grid_for(8 * (ge - gb), 256), 256, 0, x.s>>>(h->e, h->f, h->mask, h->nbr, gb, ge,
                                                                    ldexp(1.0, -2 * m), h->r);
    RG_TRY(launch_status("level multigrid coarse residual"));
    const int64_t cb = 8 * h->mg_begin[m - 1], ce = 8 * h->mg_begin[m];
    RG_TRY(fill(h->f, cb, ce, 0.0, x.s));
    k_restrict8<<<grid_for(ge - gb, 256), 256, 0, x.s>>>(h->r, h->father, gb, ge, h->f);
    RG_TRY(launch_status("level multigrid restrict"));
    RG_TRY(fill(h->e, cb, ce, 0.0, x.s));
    RG_TRY(vcoarse(x, m - 1));
    k_prolong_coarse<<<grid_for(8 * (ge - gb), 256), 256, 0, x.s>>>(h->e, h->mask, h->nbr, h->father, gb, ge);
    RG_TRY(launch_status("level multigrid coarse prolong"));
    return coarse_smooth(x, m, x.nu2);
}

rg_status vfine(const Ctx &x)
{
    rg_mg_level *h = x.h;
    const int L = h->level;
    if (L == h->lcoarse) return fine_smooth(x, x.ncoarse);
    RG_TRY(fine_smooth(x, x.nu1));
    const int64_t ob = h->fine_begin, oe = ob + h->n_fine;
    k_fine_residual<<<grid_for(8 * h->n_fine, 256), 256, 0, x.s>>>(x.phi, x.f, x.t->d_nbr27, x.t->d_father_cell, ob,
                                                                  oe, ldexp(1.0, -2 * L), h->rfine, ob);
    RG_TRY(launch_status("level multigrid residual"));
    const int64_t cb = 8 * h->mg_begin[L - 1], ce = 8 * h->mg_begin[L];
    RG_TRY(fill(h->f, cb, ce, 0.0, x.s));
    k_restrict8<<<grid_for(h->n_fine, 256), 256, 0, x.s>>>(h->rfine, h->fine_father, 0, h->n_fine, h->f);
    RG_TRY(launch_status("level multigrid restrict"));
    RG_TRY(fill(h->e, cb, ce, 0.0, x.s));
    RG_TRY(vcoarse(x, L - 1));
    k_prolong_fine<<<grid_for(8 * h->n_fine, 256), 256, 0, x.s>>>(x.phi, h->e, h->nbr, h->fine_father, ob,
                                                                 h->n_fine);
    RG_TRY(launch_status("level multigrid prolong"));
    return fine_smooth(x, x.nu2);
}

rg_status check_level(const rg_mg_level *h, const rg_tree *t)
{
    RG_REQUIRE(h && t, "null handle or tree");
    RG_REQUIRE(t->n_oct == h->tree_n_oct && t->level_begin[h->level] == h->fine_begin &&
                   t->level_begin[h->level + 1] - t->level_begin[h->level] == h->n_fine,
               "the tree changed since the hierarchy of level %d was built", h->level);
    RG_REQUIRE(t->d_nbr27 && t->d_father_cell, "tree without neighbour lists");
    return RG_OK;
}

struct TempBufs {
    std::vector<void *> p;
    ~TempBufs()
    {
        for (void *q : p) (void)hipFree(q);
    }
    rg_status alloc(void **out, size_t bytes)
    {
        *out = nullptr;
        hipError_t e = hipMalloc(out, bytes < 256 ? 256 : bytes);
        if (e != hipSuccess) return fail(RG_EHIP, "level multigrid scratch: %s", hipGetErrorString(e));
        p.push_back(*out);
        return RG_OK;
    }
};

}  // namespace
}  // namespace rg

using namespace rg;

extern "C" {

rg_status rg_mg_level_create(const rg_tree *t, int level, int lcoarse, rg_mg_level **out, void *stream)
{
    RG_REQUIRE(out, "null output handle");
    *out = nullptr;
    RG_REQUIRE(t && t->d_keys && t->d_nbr27 && t->d_father_cell, "tree without keys or neighbour lists");
    RG_REQUIRE(t->bc == RG_BC_PERIODIC, "the level multigrid needs a periodic tree");
    RG_REQUIRE(level >= t->lmin && level <= t->lmax && level <= RG_MAX_LEVEL, "level %d not in the tree", level);
    RG_REQUIRE(lcoarse >= 1 && lcoarse <= level, "coarsest level %d outside 1..%d", lcoarse, level);
    const int64_t fb = t->level_begin[level], n_fine = t->level_begin[level + 1] - fb;
    RG_REQUIRE(n_fine > 0, "level %d holds no octs", level);
    RG_REQUIRE(n_fine <= (int64_t(1) << 28), "level too large");
    hipStream_t s = as_stream(stream);
    TempBufs tmp;
    // coarse octs level by level: parents of the finer list, deduplicated
    // (K >> 3 keeps key order, so equal parents are adjacent)
    std::vector<uint64_t *> lists(RG_MAX_LEVEL + 2, nullptr);
    std::vector<int64_t> counts(RG_MAX_LEVEL + 2, 0);
    const uint64_t *prev = t->d_keys + fb;
    int64_t nprev = n_fine;
    uint64_t *shifted = nullptr;
    int64_t *d_count = nullptr;
    RG_TRY(tmp.alloc(reinterpret_cast<void **>(&shifted), size_t(n_fine) * sizeof(uint64_t)));
    RG_TRY(tmp.alloc(reinterpret_cast<void **>(&d_count), sizeof(int64_t)));
    size_t cub_bytes = 0;
    hipcub::DeviceSelect::Unique(nullptr, cub_bytes, static_cast<const uint64_t *>(nullptr),
                                 static_cast<uint64_t *>(nullptr), static_cast<int64_t *>(nullptr),
                                 static_cast<int>(n_fine), s);
    void *cub_tmp = nullptr;
    RG_TRY(tmp.alloc(&cub_tmp, cub_bytes));
    for (int m = level - 1; m >= lcoarse; --m) {
        k_shift3<<<grid_for(nprev, 256), 256, 0, s>>>(prev, nprev, shifted);
        RG_TRY(launch_status("level multigrid parent keys"));
        RG_TRY(tmp.alloc(reinterpret_cast<void **>(&lists[m]), size_t(nprev) * sizeof(uint64_t)));
        size_t cb = cub_bytes;
        if (hipcub::DeviceSelect::Unique(cub_tmp, cb, shifted, lists[m], d_count, static_cast<int>(nprev), s) !=
            hipSuccess)
            return fail(RG_EHIP, "level multigrid: unique parents");
        int64_t c = 0;
        hipError_t e = hipMemcpyAsync(&c, d_count, sizeof(c), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(RG_EHIP, "level multigrid: parent count: %s", hipGetErrorString(e));
        counts[m] = c;
        prev = lists[m];
        nprev = c;
    }
    rg_mg_level *h = new rg_mg_level();
    h->level = level;
    h->lcoarse = lcoarse;
    h->fine_begin = fb;
    h->n_fine = n_fine;
    h->tree_n_oct = t->n_oct;
    int64_t n_mg = 0;
    for (int m = 0; m <= RG_MAX_LEVEL + 1; ++m) {
        h->mg_begin[m] = n_mg;
        if (m >= lcoarse && m < level) n_mg += counts[m];
    }
    h->n_mg = n_mg;
    const size_t hash_bytes = rg_hash_workspace_bytes(n_mg);
    const size_t nm = static_cast<size_t>(n_mg);
    const size_t bytes = al256(nm * 8) + al256(nm * 27 * 4) + al256(nm * 4) + al256(size_t(n_fine) * 4) +
                         4 * al256(nm * 8 * 8) + al256(size_t(n_fine) * 8 * 8) + al256(hash_bytes);
    hipError_t e = hipMalloc(&h->mem, bytes);
    if (e != hipSuccess) {
        delete h;
        return fail(RG_EHIP, "level multigrid hierarchy: %s", hipGetErrorString(e));
    }
    char *p = static_cast<char *>(h->mem);
    auto take = [&](size_t b) {
        char *q = p;
        p += al256(b);
        return q;
    };
    h->keys = reinterpret_cast<uint64_t *>(take(nm * 8));
    h->nbr = reinterpret_cast<int32_t *>(take(nm * 27 * 4));
    h->father = reinterpret_cast<int32_t *>(take(nm * 4));
    h->fine_father = reinterpret_cast<int32_t *>(take(size_t(n_fine) * 4));
    h->e = reinterpret_cast<double *>(take(nm * 64));
    h->f = reinterpret_cast<double *>(take(nm * 64));
    h->r = reinterpret_cast<double *>(take(nm * 64));
    h->mask = reinterpret_cast<double *>(take(nm * 64));
    h->rfine = reinterpret_cast<double *>(take(size_t(n_fine) * 64));
    h->hash_ws = take(hash_bytes);
    rg_status st = RG_OK;
    for (int m = lcoarse; m < level && st == RG_OK; ++m)
        if (counts[m] > 0) {
            e = hipMemcpyAsync(h->keys + h->mg_begin[m], lists[m], size_t(counts[m]) * 8, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) st = fail(RG_EHIP, "level multigrid keys: %s", hipGetErrorString(e));
        }
    if (st == RG_OK && n_mg > 0) st = rg_hash_build(h->keys, n_mg, h->hash_ws, hash_bytes, stream);
    if (st == RG_OK && n_mg > 0) {
        HashView hv = hash_view(h->hash_ws, hash_capacity(n_mg));
        k_coarse_links<<<grid_for(n_mg, 256), 256, 0, s>>>(h->keys, n_mg, hv, lcoarse, h->nbr, h->father);
        st = launch_status("level multigrid links");
        if (st == RG_OK) {
            k_fine_links<<<grid_for(n_fine, 256), 256, 0, s>>>(t->d_keys + fb, n_fine, hv, h->fine_father);
            st = launch_status("level multigrid fine links");
        }
        // masks, finest coarse level first
        if (st == RG_OK) st = fill(h->mask, 0, 8 * n_mg, -1.0, s);
        if (st == RG_OK) {
            k_mask_level_above_fine<<<grid_for(n_fine, 256), 256, 0, s>>>(h->fine_father, n_fine, h->mask);
            st = launch_status("level multigrid masks");
        }
        for (int m = level - 2; m >= lcoarse && st == RG_OK; --m) {
            const int64_t gb = h->mg_begin[m + 1], ge = h->mg_begin[m + 2];
            k_restrict8<<<grid_for(ge - gb, 256), 256, 0, s>>>(h->mask, h->father, gb, ge, h->mask);
            st = launch_status("level multigrid masks");
        }
        if (st == RG_OK) st = fill(h->e, 0, 8 * n_mg, 0.0, s);
    }
    if (st == RG_OK) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(RG_EHIP, "level multigrid build: %s", hipGetErrorString(e));
    }
    if (st != RG_OK) {
        (void)hipFree(h->mem);
        delete h;
        return st;
    }
    *out = h;
    return RG_OK;
}

rg_status rg_mg_level_counts(const rg_mg_level *h, int64_t *h_octs)
{
    RG_REQUIRE(h && h_octs, "null pointer");
    for (int m = 0; m <= RG_MAX_LEVEL; ++m)
        h_octs[m] = (m >= h->lcoarse && m < h->level) ? h->mg_begin[m + 1] - h->mg_begin[m]
                                                      : (m == h->level ? h->n_fine : 0);
    return RG_OK;
}

rg_status rg_mg_level_vcycles(rg_mg_level *h, const rg_tree *t, double *d_phi, const double *d_f, int nu1, int nu2,
                              int ncoarse, int ncycles, void *stream)
{
    RG_TRY(check_level(h, t));
    RG_REQUIRE(d_phi && d_f, "null pointer");
    RG_REQUIRE(nu1 >= 0 && nu2 >= 0 && ncoarse >= 0 && ncycles >= 0, "negative sweep or cycle count");
    Ctx x;
    x.t = t;
    x.h = h;
    x.phi = d_phi;
    x.f = d_f;
    x.nu1 = nu1;
    x.nu2 = nu2;
    x.ncoarse = ncoarse;
    x.s = as_stream(stream);
    for (int c = 0; c < ncycles; ++c) RG_TRY(vfine(x));
    return RG_OK;
}

rg_status rg_mg_level_residual(const rg_mg_level *h, const rg_tree *t, const double *d_phi, const double *d_f,
                               double *d_r, void *stream)
{
    RG_TRY(check_level(h, t));
    RG_REQUIRE(d_phi && d_f && d_r, "null pointer");
    const int64_t ob = h->fine_begin, oe = ob + h->n_fine;
    k_fine_residual<<<grid_for(8 * h->n_fine, 256), 256, 0, as_stream(stream)>>>(
        d_phi, d_f, t->d_nbr27, t->d_father_cell, ob, oe, ldexp(1.0, -2 * h->level), d_r, 0);
    return launch_status("rg_mg_level_residual");
}

rg_status rg_mg_level_destroy(rg_mg_level *h)
{
    if (!h) return RG_OK;
    if (h->mem) (void)hipFree(h->mem);
    delete h;
    return RG_OK;
}

}  // extern "C"

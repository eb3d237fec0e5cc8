// rg_refine.hip -- refinement and de-refinement of the oct tree on the device.
//
// Paper Sec. 2.2: every step the tree changes in four stages: new octs under
// flagged cells, removal of the children of split cells that are no longer
// flagged, a bucket sort by level and a Hilbert sort inside each level (one
// radix sort of the level-major Hilbert keys here).  The paper does not give
// the criterion or the grading rule; the ones used (density threshold or
// density jump across a face; a flagged cell needs its 26 neighbours at its
// own level, which flags the coarser cells under them, finest level first)
// are restated in the header next to rg_refine.
//
// Everything runs on the device with the tree's own neighbour lists: the
// criterion reads the six face neighbours through the 27-entry list, the
// closure marks father cells through it (a missing neighbour oct's entry is
// already the coarse cell under it), and the new oct list comes from a scan
// over per-oct counts.  The host reads back two numbers (the new oct count
// and the level ranges).
#include <hipcub/hipcub.hpp>

#include "rg_internal.hpp"

namespace rg {

size_t nbr_lists_ws_bytes(int64_t n);
rg_status nbr_lists_device(const uint64_t *d_keys, int64_t n, const int64_t *h_level_begin, int lmin, int lmax,
                           void *d_ws, size_t ws_bytes, const int32_t **list, int64_t *nbricks, int64_t *nrest,
                           hipStream_t s);

namespace {

constexpr int NVR = 5;   // conserved variables per cell

__device__ __forceinline__ int face_slot(int side)
{
    // x-, x+, y-, y+, z-, z+ in the (dx+1) + 3(dy+1) + 9(dz+1) numbering
    return side == 0 ? 12 : side == 1 ? 14 : side == 2 ? 10 : side == 3 ? 16 : side == 4 ? 4 : 22;
}

struct CritArgs {
    const double *u;
    const int32_t *nbr27;
    int64_t ob, oe;       // octs of the levels that may be flagged
    double rho_thresh, grad_thresh;
    uint32_t *flags;
    int whole;            // widen a flag to all 8 cells of its oct (4^3-cell blocks)
};

// one thread per cell: the criterion on the cell's density and its six face
// neighbours' (same-level cell, else the coarse cell under the missing oct,
// outside: the cell itself).  Launched with a multiple of 64 threads per
// block, so an oct's eight cells sit in one wave.
__global__ void k_refine_criterion(CritArgs a)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t o = a.ob + (t >> 3);
    if (o >= a.oe) return;
    const int c = static_cast<int>(t & 7);
    const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
    const double rc = a.u[NVR * (8 * o + c)];
    bool flag = a.rho_thresh > 0.0 && rc > a.rho_thresh;
    if (a.grad_thresh > 0.0) {
        for (int side = 0; side < 6; ++side) {
            int p[3] = {cx, cy, cz};
            const int ax = side >> 1;
            p[ax] += (side & 1) ? 1 : -1;
            double rn;
            if (p[ax] >= 0 && p[ax] <= 1) {
                rn = a.u[NVR * (8 * o + p[0] + 2 * p[1] + 4 * p[2])];
            } else {
                const int32_t e = a.nbr27[27 * o + face_slot(side)];
                if (e == RG_NBR_OUTSIDE) {
                    rn = rc;
                } else if (e >= 0) {
                    const int q[3] = {p[0] & 1, p[1] & 1, p[2] & 1};
                    rn = a.u[NVR * (8 * int64_t(e) + q[0] + 2 * q[1] + 4 * q[2])];
                } else {
                    rn = a.u[NVR * (-1 - int64_t(e))];
                }
            }
            const double d = fabs(rn - rc) / (rn + rc);
            flag = flag || d > a.grad_thresh;
        }
    }
    // the eight lanes of an oct are eight consecutive lanes of one wave
    const uint64_t votes = __ballot(flag);
    const int lane = threadIdx.x & 63;
    uint32_t m = static_cast<uint32_t>((votes >> (lane & ~7)) & 0xffu);
    if (a.whole && m) m = 0xffu;
    if (c == 0) a.flags[o] = m;
}

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// one thread per oct of one level: a flagged cell marks the father cell of
// every level-l oct holding one of its 26 neighbours or itself.  A cell with
// in-oct position c reaches, along each axis, its own oct and the neighbour
// oct on its side (offset -1 for c = 0, +1 for c = 1), so the oct's flagged
// cells need at most 27 neighbour octs; each target bit is set by an atomic
// only if a plain read does not already show it (many octs mark the same
// coarse cells).
__global__ void k_refine_closure(const int32_t *__restrict__ nbr27, const int32_t *__restrict__ father,
                                 int64_t ob, int64_t oe, uint32_t *flags, int whole)
{
    const int64_t o = ob + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= oe) return;
    const uint32_t m = flags[o] & 0xffu;
    if (!m) return;
    uint32_t need = 0;   // bit (sx+1) + 3(sy+1) + 9(sz+1): neighbour oct offsets needed
    for (int c = 0; c < 8; ++c) {
        if (!((m >> c) & 1u)) continue;
        const int ox = (c & 1) ? 1 : -1, oy = ((c >> 1) & 1) ? 1 : -1, oz = (c >> 2) ? 1 : -1;
        for (int b = 0; b < 8; ++b) {
            const int sx = (b & 1) ? ox : 0, sy = ((b >> 1) & 1) ? oy : 0, sz = (b >> 2) ? oz : 0;
            need |= 1u << ((sx + 1) + 3 * (sy + 1) + 9 * (sz + 1));
        }
    }
    for (int slot = 0; slot < 27; ++slot) {
        if (!((need >> slot) & 1u)) continue;
        const int32_t e = nbr27[27 * o + slot];
        if (e == RG_NBR_OUTSIDE) continue;
        const int64_t fc = e >= 0 ? int64_t(father[e]) : (-1 - int64_t(e));
        if (fc < 0) continue;   // coarsest level: nothing to mark
        const uint32_t bit = whole ? 0xffu : 1u << (fc & 7);
        if ((flags[fc >> 3] & bit) != bit) atomicOr(&flags[fc >> 3], bit);
    }
}

__device__ __forceinline__ bool kept(const uint32_t *flags, const int32_t *father, int64_t o, bool coarsest)
{
    if (coarsest) return true;
    const int32_t f = father[o];
    return f >= 0 && ((flags[f >> 3] >> (f & 7)) & 1u);
}

// per oct: 1 if kept, plus one per flagged leaf cell (its new child)
__global__ void k_refine_count(const uint32_t *__restrict__ flags, const int32_t *__restrict__ father,
                               const uint32_t *__restrict__ son, int64_t n, int64_t coarse_end, int32_t *cnt)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const bool k = kept(flags, father, o, o < coarse_end);
    cnt[o] = k ? 1 + __popc(flags[o] & ~son[o] & 0xffu) : 0;
}

__global__ void k_refine_emit(const uint32_t *__restrict__ flags, const int32_t *__restrict__ father,
                              const uint32_t *__restrict__ son, const int32_t *__restrict__ ijkl, int64_t n,
                              int64_t coarse_end, const int32_t *__restrict__ off, int32_t *new_ijkl, int32_t *src)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    if (!kept(flags, father, o, o < coarse_end)) return;
    int64_t m = off[o];
    const int32_t i = ijkl[4 * o], j = ijkl[4 * o + 1], k = ijkl[4 * o + 2], l = ijkl[4 * o + 3];
    new_ijkl[4 * m] = i;
    new_ijkl[4 * m + 1] = j;
    new_ijkl[4 * m + 2] = k;
    new_ijkl[4 * m + 3] = l;
    src[m] = static_cast<int32_t>(o);
    ++m;
    const uint32_t fresh = flags[o] & ~son[o] & 0xffu;
    for (int c = 0; c < 8; ++c) {
        if (!((fresh >> c) & 1u)) continue;
        new_ijkl[4 * m] = 2 * i + (c & 1);
        new_ijkl[4 * m + 1] = 2 * j + ((c >> 1) & 1);
        new_ijkl[4 * m + 2] = 2 * k + (c >> 2);
        new_ijkl[4 * m + 3] = l + 1;
        src[m] = static_cast<int32_t>(-1 - (8 * o + c));
        ++m;
    }
}

// sorted position p: coordinates and state from emitted entry perm[p]; a kept
// oct copies its 8 cells, a new one repeats its father cell
__global__ void k_refine_gather(const int32_t *__restrict__ perm, const int32_t *__restrict__ new_ijkl,
                                const int32_t *__restrict__ src, const double *__restrict__ u, int64_t m,
                                int32_t *ijkl_out, double *u_out)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t p = t / 40;
    const int r = static_cast<int>(t - 40 * p);
    if (p >= m) return;
    const int32_t e = perm[p];
    const int32_t s = src[e];
    if (r < 4) ijkl_out[4 * p + r] = new_ijkl[4 * int64_t(e) + r];
    const double v = s >= 0 ? u[40 * int64_t(s) + r] : u[NVR * (-1 - int64_t(s)) + (r % NVR)];
    u_out[40 * p + r] = v;
}

struct RefineWs {
    uint32_t *flags;
    int32_t *cnt, *off, *src, *new_ijkl, *total;
    void *temp;
    size_t temp_bytes;
};

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

size_t scan_temp_bytes(int64_t cap)
{
    size_t temp = 0;
    hipcub::DeviceScan::ExclusiveSum(nullptr, temp, static_cast<const int32_t *>(nullptr),
                                     static_cast<int32_t *>(nullptr), static_cast<int>(cap > 0 ? cap : 1));
    return temp;
}

RefineWs carve(void *ws, int64_t cap)
{
    char *p = static_cast<char *>(ws);
    RefineWs w;
    w.flags = reinterpret_cast<uint32_t *>(p);
    p += al256(4 * cap);
    w.cnt = reinterpret_cast<int32_t *>(p);
    p += al256(4 * cap);
    w.off = reinterpret_cast<int32_t *>(p);
    p += al256(4 * cap);
    w.src = reinterpret_cast<int32_t *>(p);
    p += al256(4 * cap);
    w.new_ijkl = reinterpret_cast<int32_t *>(p);
    p += al256(16 * cap);
    w.total = reinterpret_cast<int32_t *>(p);
    p += 256;
    w.temp = p;
    w.temp_bytes = al256(scan_temp_bytes(cap));
    return w;
}

rg_status check_tree(const rg_tree *t, const rg_refine_params *pr)
{
    RG_REQUIRE(t && pr, "null pointer");
    RG_REQUIRE(t->n_oct > 0 && t->lmin >= 1 && t->lmax >= t->lmin && t->lmax <= RG_MAX_LEVEL, "bad tree");
    RG_REQUIRE(t->level_begin[t->lmin] == 0 && t->level_begin[t->lmax + 1] == t->n_oct, "bad level ranges");
    RG_REQUIRE(t->d_nbr27 && t->d_father_cell && t->d_son_mask, "tree without neighbour lists");
    RG_REQUIRE(pr->lmax >= t->lmin && pr->lmax <= RG_MAX_LEVEL, "refinement level limit %d out of range", pr->lmax);
    RG_REQUIRE(pr->nsubgrid == 0 || pr->nsubgrid == 2 || pr->nsubgrid == 4, "nsubgrid %d not 2 or 4", pr->nsubgrid);
    return RG_OK;
}

// criterion, then (if closure) the grading closure from the finest level down
rg_status flags_pass(const rg_tree *t, const double *d_u, const rg_refine_params *pr, int closure, uint32_t *flags,
                     hipStream_t s)
{
    k_zero_u32<<<grid_for(t->n_oct, 256), 256, 0, s>>>(flags, t->n_oct);
    RG_TRY(launch_status("refine flags clear"));
    const int ltop = t->lmax < pr->lmax - 1 ? t->lmax : pr->lmax - 1;
    if (ltop >= t->lmin) {
        CritArgs a;
        a.u = d_u;
        a.nbr27 = t->d_nbr27;
        a.ob = 0;
        a.oe = t->level_begin[ltop + 1];
        a.rho_thresh = pr->rho_thresh;
        a.grad_thresh = pr->grad_thresh;
        a.flags = flags;
        a.whole = pr->nsubgrid == 4;
        if (a.oe > 0) {
            k_refine_criterion<<<grid_for(8 * a.oe, 256), 256, 0, s>>>(a);
            RG_TRY(launch_status("refine criterion"));
        }
    }
    if (closure) {
        for (int l = t->lmax; l > t->lmin; --l) {
            const int64_t ob = t->level_begin[l], oe = t->level_begin[l + 1];
            if (oe <= ob) continue;
            k_refine_closure<<<grid_for(oe - ob, 256), 256, 0, s>>>(t->d_nbr27, t->d_father_cell, ob, oe, flags,
                                                                    pr->nsubgrid == 4);
            RG_TRY(launch_status("refine closure"));
        }
    }
    return RG_OK;
}

}  // namespace
}  // namespace rg

using namespace rg;

extern "C" {

size_t rg_refine_workspace_bytes(int64_t capacity)
{
    const int64_t cap = capacity > 0 ? capacity : 1;
    const size_t core = 4 * al256(4 * cap) + al256(16 * cap) + 256 + al256(scan_temp_bytes(cap)) + 256;
    return core + al256(nbr_lists_ws_bytes(cap));
}

rg_status rg_refine_flags(const rg_tree *t, const double *d_u, const rg_refine_params *p, int closure,
                          uint32_t *d_flags, void *stream)
{
    RG_TRY(check_tree(t, p));
    RG_REQUIRE(d_u && d_flags, "null pointer");
    return flags_pass(t, d_u, p, closure, d_flags, as_stream(stream));
}

rg_status rg_refine(rg_tree *t, const double *d_u, double *d_u_new, const rg_refine_params *p, void *d_ws,
                    size_t ws_bytes, void *stream)
{
    RG_TRY(check_tree(t, p));
    RG_REQUIRE(d_u && d_u_new && d_ws, "null pointer");
    RG_REQUIRE(d_u != d_u_new, "state buffers must not alias");
    RG_REQUIRE(t->d_ijkl && t->d_keys_scratch && t->d_perm && t->d_sort_ws && t->d_level_begin && t->d_hash_ws,
               "refinement needs coordinates, scratch keys, permutation, sort workspace, level ranges and hash "
               "workspace");
    const int64_t cap = t->capacity > 0 ? t->capacity : t->n_oct;
    RG_REQUIRE(cap >= t->n_oct && cap <= (int64_t(1) << 28), "capacity %lld below the oct count",
               static_cast<long long>(cap));
    RG_REQUIRE(ws_bytes >= rg_refine_workspace_bytes(cap) && aligned(d_ws, 256), "refine workspace too small");
    RG_REQUIRE(t->sort_ws_bytes >= rg_sort_workspace_bytes(cap), "sort workspace below capacity");
    RG_REQUIRE(t->hash_ws_bytes >= rg_hash_workspace_bytes(cap), "hash workspace below capacity");
    hipStream_t s = as_stream(stream);
    const int64_t n = t->n_oct;
    RefineWs w = carve(d_ws, cap);
    RG_TRY(flags_pass(t, d_u, p, 1, w.flags, s));
    const int64_t coarse_end = t->level_begin[t->lmin + 1];
    k_refine_count<<<grid_for(n, 256), 256, 0, s>>>(w.flags, t->d_father_cell, t->d_son_mask, n, coarse_end, w.cnt);
    RG_TRY(launch_status("refine count"));
    size_t tb = w.temp_bytes;
    if (hipcub::DeviceScan::ExclusiveSum(w.temp, tb, w.cnt, w.off, static_cast<int>(n), s) != hipSuccess)
        return fail(RG_EHIP, "refine scan");
    int32_t h_last[2] = {0, 0};
    if (hipMemcpyAsync(&h_last[0], w.off + (n - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&h_last[1], w.cnt + (n - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(RG_EHIP, "refine count readback");
    const int64_t m = int64_t(h_last[0]) + h_last[1];
    if (m > cap)
        return fail(RG_EFULL, "refined tree needs %lld octs, capacity %lld", static_cast<long long>(m),
                    static_cast<long long>(cap));
    k_refine_emit<<<grid_for(n, 256), 256, 0, s>>>(w.flags, t->d_father_cell, t->d_son_mask, t->d_ijkl, n,
                                                   coarse_end, w.off, w.new_ijkl, w.src);
    RG_TRY(launch_status("refine emit"));
    // stage 3-4: keys of the new octs, one radix sort (level-major, Hilbert inside a level)
    const int lnew = t->lmax + 1 < p->lmax ? t->lmax + 1 : p->lmax;
    RG_TRY(rg_encode_keys(w.new_ijkl, m, t->d_keys_scratch, stream));
    RG_TRY(sort_keys_bits(t->d_keys_scratch, m, t->d_keys, t->d_perm, t->d_sort_ws, t->sort_ws_bytes, 3 * lnew, s));
    k_refine_gather<<<grid_for(40 * m, 256), 256, 0, s>>>(t->d_perm, w.new_ijkl, w.src, d_u, m,
                                                         t->d_ijkl, d_u_new);
    RG_TRY(launch_status("refine gather"));
    RG_TRY(rg_level_ranges(t->d_keys, m, t->d_level_begin, stream));
    int64_t lb[RG_MAX_LEVEL + 2];
    if (hipMemcpyAsync(lb, t->d_level_begin, sizeof(lb), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(RG_EHIP, "refine level readback");
    int lmax = t->lmin;
    for (int l = t->lmin; l <= RG_MAX_LEVEL; ++l)
        if (lb[l + 1] > lb[l]) lmax = l;
    for (int l = 0; l < RG_MAX_LEVEL + 2; ++l) t->level_begin[l] = lb[l];
    t->n_oct = m;
    t->lmax = lmax;
    t->sched = nullptr;
    RG_TRY(rg_hash_build(t->d_keys, m, t->d_hash_ws, t->hash_ws_bytes, stream));
    // neighbour lists brick by brick: the complete bricks follow from the keys
    const size_t core = 4 * al256(4 * cap) + al256(16 * cap) + 256 + al256(scan_temp_bytes(cap)) + 256;
    const int32_t *lst = nullptr;
    int64_t nb = 0, nr = 0;
    RG_TRY(nbr_lists_device(t->d_keys, m, t->level_begin, t->lmin, t->lmax, static_cast<char *>(d_ws) + core,
                            ws_bytes - core, &lst, &nb, &nr, s));
    return neighbours_scheduled(t->d_hash_ws, t->d_keys, m, t->lmin, t->lmax, t->level_begin[t->lmax], t->bc, lst,
                                nb, lst + nb, nr, t->d_nbr27, t->d_father_cell, t->d_son_mask, s);
}

}  // extern "C"

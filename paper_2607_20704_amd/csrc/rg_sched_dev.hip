// rg_sched_dev.hip -- the kernel schedule built on the device.
//
// Same lists as rg_schedule_build (per level: complete Hilbert-aligned
// 8^3-oct bricks that border no coarse cell, the other octs; every complete
// brick and the other octs for the neighbour build; per level above lmin the
// octs with a coarse cell across a face; per level the complete sibling
// groups outside the bricks and the octs outside bricks and groups), found
// without copying the tree to the host: one pass marks complete bricks and
// the bricks that touch a coarse cell, a second pass evaluates the seven
// membership tests per oct, seven scans give every oct its place, and a
// scatter writes the lists in key order.  The host reads back only the
// per-level list lengths.  A tree that changes every step (refinement) keeps
// its brick kernel this way.
#include <hipcub/hipcub.hpp>

#include "rg_internal.hpp"

namespace rg {
namespace {

// bricks, per-oct, all complete bricks, octs outside them, border octs,
// sibling groups, octs outside bricks and groups
constexpr int kLists = 7;
constexpr int64_t kBrick = 512;      // octs per brick
constexpr int64_t kGroup = 8;        // octs per sibling group
constexpr int kLB = RG_MAX_LEVEL + 2;

struct SchedArgs {
    const uint64_t *keys;
    const int32_t *nbr27;
    int64_t n;
    int64_t begin[kLB];
    int lmin;
};

__device__ __forceinline__ int level_of(const SchedArgs &a, int64_t o)
{
    int l = a.lmin;
    while (l < RG_MAX_LEVEL && o >= a.begin[l + 1]) ++l;
    return l;
}

// first oct of the complete brick holding o, or -1
__device__ __forceinline__ int64_t brick_first(const SchedArgs &a, int64_t o, int l)
{
    const uint64_t k = a.keys[o];
    const int64_t r = static_cast<int64_t>(k & uint64_t(kBrick - 1));
    const int64_t f = o - r;
    if (f < a.begin[l] || f + kBrick - 1 >= a.begin[l + 1]) return -1;
    if (a.keys[f] != k - uint64_t(r) || a.keys[f + kBrick - 1] != k - uint64_t(r) + uint64_t(kBrick - 1)) return -1;
    return f;
}

// first oct of the complete sibling group holding o (levels above lmin), or -1
__device__ __forceinline__ int64_t group_first(const SchedArgs &a, int64_t o, int l)
{
    if (l <= a.lmin) return -1;
    const uint64_t k = a.keys[o];
    const int64_t r = static_cast<int64_t>(k & uint64_t(kGroup - 1));
    const int64_t f = o - r;
    if (f < a.begin[l] || f + kGroup - 1 >= a.begin[l + 1]) return -1;
    if (a.keys[f] != k - uint64_t(r) || a.keys[f + kGroup - 1] != k - uint64_t(r) + uint64_t(kGroup - 1)) return -1;
    return f;
}

__device__ __forceinline__ bool coarse_entry(int32_t v) { return v < 0 && v != RG_NBR_OUTSIDE; }

__global__ void k_sched_zero(uint32_t *p, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// a complete brick with a coarse entry anywhere in its octs' lists is marked
__global__ void k_sched_mark(SchedArgs a, uint32_t *bad)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= a.n) return;
    const int l = level_of(a, o);
    const int64_t f = brick_first(a, o, l);
    if (f < 0) return;
    bool coarse = false;
    for (int j = 0; j < 27; ++j) coarse = coarse || coarse_entry(a.nbr27[27 * o + j]);
    if (coarse) atomicOr(&bad[f], 1u);
}

__global__ void k_sched_pred(SchedArgs a, const uint32_t *__restrict__ bad, int32_t *pred)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= a.n) return;
    const int l = level_of(a, o);
    const int64_t f = brick_first(a, o, l);
    const bool complete = f >= 0;
    const bool covered = complete && bad[f] == 0;
    bool border = false;
    if (l > a.lmin) {
        const int slots[6] = {12, 14, 10, 16, 4, 22};
        for (int s = 0; s < 6; ++s) border = border || coarse_entry(a.nbr27[27 * o + slots[s]]);
    }
    pred[0 * a.n + o] = covered && f == o;
    pred[1 * a.n + o] = !covered;
    pred[2 * a.n + o] = complete && f == o;
    pred[3 * a.n + o] = !complete;
    pred[4 * a.n + o] = border;
    const int64_t g = covered ? -1 : group_first(a, o, l);
    pred[5 * a.n + o] = g >= 0 && g == o;
    pred[6 * a.n + o] = !covered && g < 0;
}

// per list and level boundary: the number of list members before the
// boundary (the last boundary gives the list's length)
__global__ void k_sched_bounds(SchedArgs a, const int32_t *__restrict__ pred, const int32_t *__restrict__ pos,
                               int64_t *out)
{
    const int t = threadIdx.x;
    if (t >= kLists * kLB) return;
    const int k = t / kLB, l = t - kLB * k;
    const int64_t b = a.begin[l] < a.n ? a.begin[l] : a.n;
    const int32_t *p = pos + int64_t(k) * a.n;
    const int32_t *q = pred + int64_t(k) * a.n;
    out[t] = b < a.n ? int64_t(p[b]) : int64_t(p[a.n - 1]) + q[a.n - 1];
}

struct Bases {
    int64_t base[kLists];
};

__global__ void k_sched_scatter(int64_t n, const int32_t *__restrict__ pred, const int32_t *__restrict__ pos,
                                Bases b, int32_t *list)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
#pragma unroll
    for (int k = 0; k < kLists; ++k)
        if (pred[int64_t(k) * n + o]) list[b.base[k] + pos[int64_t(k) * n + o]] = static_cast<int32_t>(o);
}

// keys only: first octs of complete bricks (pred[0]) and octs outside
// complete bricks (pred[1]), for the brick-wise neighbour build
__global__ void k_nbr_pred(SchedArgs a, int32_t *pred)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= a.n) return;
    const int64_t f = brick_first(a, o, level_of(a, o));
    pred[o] = f >= 0 && f == o;
    pred[a.n + o] = f < 0;
}

__global__ void k_nbr_scatter(int64_t n, const int32_t *__restrict__ pred, const int32_t *__restrict__ pos,
                              int64_t base1, int32_t *list)
{
    const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    if (pred[o]) list[pos[o]] = static_cast<int32_t>(o);
    if (pred[n + o]) list[base1 + pos[n + o]] = static_cast<int32_t>(o);
}

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

size_t scan_bytes(int64_t n)
{
    size_t temp = 0;
    hipcub::DeviceScan::ExclusiveSum(nullptr, temp, static_cast<const int32_t *>(nullptr),
                                     static_cast<int32_t *>(nullptr), static_cast<int>(n > 0 ? n : 1));
    return temp;
}

}  // namespace

size_t nbr_lists_ws_bytes(int64_t n)
{
    n = n > 0 ? n : 1;
    return 2 * al(8 * n) + al(4 * n + 4 * (n / kBrick) + 4) + al(scan_bytes(n)) + 256;
}

// The neighbour-build lists of a tree from its keys and level ranges alone
// (complete bricks, then the other octs, in key order) into the workspace;
// *list points at them.  Synchronises once for the two lengths.
rg_status nbr_lists_device(const uint64_t *d_keys, int64_t n, const int64_t *h_level_begin, int lmin, int lmax,
                           void *d_ws, size_t ws_bytes, const int32_t **list, int64_t *nbricks, int64_t *nrest,
                           hipStream_t s)
{
    RG_REQUIRE(ws_bytes >= nbr_lists_ws_bytes(n) && aligned(d_ws, 256), "neighbour-list workspace too small");
    char *p = static_cast<char *>(d_ws);
    int32_t *pred = reinterpret_cast<int32_t *>(p);
    p += al(8 * n);
    int32_t *pos = reinterpret_cast<int32_t *>(p);
    p += al(8 * n);
    int32_t *lst = reinterpret_cast<int32_t *>(p);
    p += al(4 * n + 4 * (n / kBrick) + 4);
    void *temp = p;
    SchedArgs a;
    a.keys = d_keys;
    a.nbr27 = nullptr;
    a.n = n;
    for (int l = 0; l < kLB; ++l) a.begin[l] = h_level_begin[l];
    for (int l = lmax + 1; l < kLB; ++l) a.begin[l] = n;
    a.lmin = lmin;
    k_nbr_pred<<<grid_for(n, 256), 256, 0, s>>>(a, pred);
    RG_TRY(launch_status("neighbour lists"));
    for (int k = 0; k < 2; ++k) {
        size_t tb = al(scan_bytes(n));
        if (hipcub::DeviceScan::ExclusiveSum(temp, tb, pred + k * n, pos + k * n, static_cast<int>(n), s) !=
            hipSuccess)
            return fail(RG_EHIP, "neighbour-list scan");
    }
    int32_t h[4];
    if (hipMemcpyAsync(&h[0], pos + (n - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&h[1], pred + (n - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&h[2], pos + (2 * n - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&h[3], pred + (2 * n - 1), 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(RG_EHIP, "neighbour-list readback");
    *nbricks = int64_t(h[0]) + h[1];
    *nrest = int64_t(h[2]) + h[3];
    k_nbr_scatter<<<grid_for(n, 256), 256, 0, s>>>(n, pred, pos, *nbricks, lst);
    RG_TRY(launch_status("neighbour-list scatter"));
    *list = lst;
    return RG_OK;
}

}  // namespace rg

using namespace rg;

extern "C" {

size_t rg_schedule_workspace_bytes(int64_t n_oct)
{
    const int64_t n = n_oct > 0 ? n_oct : 1;
    return al(4 * n) + 2 * al(4 * kLists * n) + al(8 * kLists * kLB) + al(scan_bytes(n)) + 256;
}

rg_status rg_schedule_build_device(const rg_tree *t, int32_t *d_list, int64_t capacity, void *d_ws, size_t ws_bytes,
                                   rg_schedule *out, void *stream)
{
    RG_REQUIRE(t && d_list && out && d_ws, "null pointer");
    RG_REQUIRE(t->n_oct > 0 && t->n_oct <= (int64_t(1) << 28) && capacity >= 4 * t->n_oct,
               "list capacity below 4 n_oct");
    RG_REQUIRE(t->lmin >= 1 && t->lmax >= t->lmin && t->lmax <= RG_MAX_LEVEL, "bad levels");
    RG_REQUIRE(t->level_begin[t->lmin] == 0 && t->level_begin[t->lmax + 1] == t->n_oct, "bad level ranges");
    RG_REQUIRE(t->d_keys && t->d_nbr27, "tree without keys or neighbour lists");
    RG_REQUIRE(ws_bytes >= rg_schedule_workspace_bytes(t->n_oct) && aligned(d_ws, 256), "workspace too small");
    const int64_t n = t->n_oct;
    hipStream_t s = as_stream(stream);
    char *p = static_cast<char *>(d_ws);
    uint32_t *bad = reinterpret_cast<uint32_t *>(p);
    p += al(4 * n);
    int32_t *pred = reinterpret_cast<int32_t *>(p);
    p += al(4 * kLists * n);
    int32_t *pos = reinterpret_cast<int32_t *>(p);
    p += al(4 * kLists * n);
    int64_t *bounds = reinterpret_cast<int64_t *>(p);
    p += al(8 * kLists * kLB);
    void *temp = p;
    const size_t temp_bytes = al(scan_bytes(n));

    SchedArgs a;
    a.keys = t->d_keys;
    a.nbr27 = t->d_nbr27;
    a.n = n;
    for (int l = 0; l < kLB; ++l) a.begin[l] = t->level_begin[l];
    for (int l = t->lmax + 1; l < kLB; ++l) a.begin[l] = n;
    a.lmin = t->lmin;
    k_sched_zero<<<grid_for(n, 256), 256, 0, s>>>(bad, n);
    RG_TRY(launch_status("schedule clear"));
    k_sched_mark<<<grid_for(n, 256), 256, 0, s>>>(a, bad);
    RG_TRY(launch_status("schedule bricks"));
    k_sched_pred<<<grid_for(n, 256), 256, 0, s>>>(a, bad, pred);
    RG_TRY(launch_status("schedule tests"));
    for (int k = 0; k < kLists; ++k) {
        size_t tb = temp_bytes;
        if (hipcub::DeviceScan::ExclusiveSum(temp, tb, pred + k * n, pos + k * n, static_cast<int>(n), s) !=
            hipSuccess)
            return fail(RG_EHIP, "schedule scan");
    }
    static_assert(kLists * kLB <= 256, "one thread per list and level");
    k_sched_bounds<<<1, 256, 0, s>>>(a, pred, pos, bounds);
    RG_TRY(launch_status("schedule bounds"));
    int64_t h[kLists * kLB];
    if (hipMemcpyAsync(h, bounds, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(RG_EHIP, "schedule readback");
    auto at = [&](int k, int l) { return h[k * kLB + l]; };
    Bases b;
    int64_t total = 0;
    for (int k = 0; k < kLists; ++k) {
        b.base[k] = total;
        total += at(k, kLB - 1);
    }
    if (total > capacity) return fail(RG_EINVAL, "schedule exceeds list capacity");
    k_sched_scatter<<<grid_for(n, 256), 256, 0, s>>>(n, pred, pos, b, d_list);
    RG_TRY(launch_status("schedule scatter"));
    for (int l = 0; l < kLB; ++l)
        out->brick_begin[l] = out->brick_count[l] = out->rest_begin[l] = out->rest_count[l] = out->border_begin[l] =
            out->border_count[l] = out->group_begin[l] = out->group_count[l] = out->single_begin[l] =
                out->single_count[l] = 0;
    for (int l = t->lmin; l <= t->lmax; ++l) {
        out->brick_begin[l] = b.base[0] + at(0, l);
        out->brick_count[l] = at(0, l + 1) - at(0, l);
        out->rest_begin[l] = b.base[1] + at(1, l);
        out->rest_count[l] = at(1, l + 1) - at(1, l);
        if (l > t->lmin) {
            out->border_begin[l] = b.base[4] + at(4, l);
            out->border_count[l] = at(4, l + 1) - at(4, l);
        }
        out->group_begin[l] = b.base[5] + at(5, l);
        out->group_count[l] = at(5, l + 1) - at(5, l);
        out->single_begin[l] = b.base[6] + at(6, l);
        out->single_count[l] = at(6, l + 1) - at(6, l);
    }
    out->nbr_brick_begin = b.base[2];
    out->nbr_brick_count = at(2, kLB - 1);
    out->nbr_rest_begin = b.base[3];
    out->nbr_rest_count = at(3, kLB - 1);
    out->d_list = d_list;
    return RG_OK;
}

}  // extern "C"

// rg_tree.hip -- oct keys, sort, hash table and neighbour lists (gfx950).
//
// Paper: an oct is the key tuple (i,j,k,l) mapped to its position in device
// memory through an fnv64 hash with linear probing (Sec. 2.1); octs are
// sorted by level and along a Hilbert curve (Sec. 2.2); father and
// neighbour index arrays are precomputed per oct for stencils, with ghost
// values where the neighbour oct does not exist (Sec. 2.3); the neighbour
// topology is a flat 27-entry list per oct built from hash lookups (Sec. 5);
// insertion claims a slot with compare-and-swap (Sec. 6; gfx950 has native
// 64-bit CAS, so the key itself is the CAS target).
#include <hipcub/hipcub.hpp>

#include <mutex>

#include "rg_internal.hpp"
#include "rg_nbr.hpp"

namespace rg {
rg_status check_sink(int64_t *h_bad_index, hipStream_t s);
namespace {

__global__ void k_fill_u32(uint32_t *d, int64_t n, uint32_t v)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

__global__ void k_fill_u64(uint64_t *d, int64_t n, uint64_t v)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

__global__ void k_encode(const int32_t *__restrict__ ijkl, int64_t n, uint64_t *__restrict__ keys)
{
    int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const int4 c = reinterpret_cast<const int4 *>(ijkl)[o];
    keys[o] = oct_key(c.x, c.y, c.z, c.w);
}

__global__ void k_decode(const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ ijkl)
{
    int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    int32_t i, j, k, l;
    key_coords(keys[o], i, j, k, l);
    reinterpret_cast<int4 *>(ijkl)[o] = make_int4(i, j, k, l);
}

__global__ void k_iota(int32_t *d, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) d[i] = static_cast<int32_t>(i);
}

// begin[l] = first position whose level is >= l; one writer per entry
__global__ void k_level_ranges(const uint64_t *__restrict__ keys, int64_t n, int64_t *__restrict__ begin)
{
    int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (o >= n) return;
    int lv = key_level(keys[o]);
    int prev = (o == 0) ? 0 : key_level(keys[o - 1]);
    if (o == 0) begin[0] = 0;
    for (int l = prev + 1; l <= lv && l <= RG_MAX_LEVEL + 1; ++l) begin[l] = o;
    if (o == n - 1)
        for (int l = lv + 1; l <= RG_MAX_LEVEL + 1; ++l) begin[l] = n;
}

__global__ void k_zero_i64(int64_t *d, int n)
{
    int i = threadIdx.x;
    if (i < n) d[i] = 0;
}

__global__ void k_permute_rows(const double *__restrict__ in, const int32_t *__restrict__ perm, int64_t rows, int rd,
                               double *__restrict__ out)
{
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= rows * rd) return;
    int64_t r = t / rd;
    int e = static_cast<int>(t - r * rd);
    out[t] = in[int64_t(perm[r]) * rd + e];
}

// clears every slot; thread 0 also resets the header
__global__ void k_hash_clear(HashHeader *hdr, uint64_t *keys, uint64_t cap, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < static_cast<int64_t>(cap)) keys[i] = 0;
    if (i == 0) {
        hdr->cap = cap;
        hdr->n = n;
        hdr->err = 0;
        hdr->bad = -1;
    }
}

__global__ void k_hash_insert(const uint64_t *__restrict__ in, int64_t n, HashHeader *hdr, uint64_t *keys,
                              int32_t *vals, uint64_t mask)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) hash_insert_one(hdr, keys, vals, mask, in[i], i);
}

// ---------------------------------------------------------------------------
// Segmented table build.  The table is cut into segments of 2^kSegLog slots.
// Keys are bucketed by the segment of their home slot (a short radix sort of
// segment numbers); one workgroup then builds each segment in LDS with LDS
// compare-and-swap and writes it out whole.  A probe sequence that runs past
// the end of its segment is finished afterwards with global compare-and-swap
// on the finished table.  Every key ends at the first free slot at or after
// its home slot at the time it is placed, so the result is a valid
// linear-probing table (slot positions depend on the placement order, as
// with any concurrent build; lookups do not).
// ---------------------------------------------------------------------------

constexpr int kSegLog = 12;
constexpr int kSegMax = 1 << kSegLog;
constexpr int kSegThreads = 512;   // threads of k_seg_build (48 KB of LDS: 3 workgroups per CU)
constexpr int kSegKpt = 6;         // its segment entries per thread per pass

struct SegBuild {
    uint64_t *bkeys;                                 // [n] the keys, bucketed by segment
    uint32_t *idx;                                   // [n] their indices, in the same order
    uint32_t *hist;                                  // [nseg][nblk] per-chunk counts, then offsets
    uint32_t *seg_begin, *seg_end, *seg_tot;         // [nseg] each
    uint32_t *ovf_count;                             // [64] (first used)
    uint32_t *ovf;                                   // [n]
    int seg_log, bits;
    int64_t nseg, nblk;
};

// keys per bucketing workgroup
constexpr int kBucketChunk = 4096;
constexpr int kBucketThreads = 1024;   // per chunk: four keys per thread
constexpr int kBucketKpt = kBucketChunk / kBucketThreads;

// The chunk of a bucketing workgroup.  Workgroup w runs on XCD w % 8; each
// XCD takes a contiguous range of chunks, so that the runs which
// neighbouring chunks write side by side in every segment's range (and in
// the count matrix) meet in one L2 and leave it as whole lines.  The grid is
// 8 ceil(nblk / 8) workgroups; those past the last chunk return at once.
__device__ __forceinline__ int64_t bucket_chunk(int64_t nblk)
{
    const int64_t per = (nblk + 7) / 8;
    return static_cast<int64_t>(blockIdx.x % 8) * per + blockIdx.x / 8;
}

inline unsigned bucket_grid(int64_t nblk) { return static_cast<unsigned>(8 * ((nblk + 7) / 8)); }

// the keys of chunk blk that this thread handles (0 past the end), loaded
// together so that the thread waits for memory once, not once per key
__device__ __forceinline__ void chunk_keys(const uint64_t *__restrict__ keys, int64_t n, int64_t blk,
                                           uint64_t (&kk)[kBucketKpt])
{
#pragma unroll
    for (int j = 0; j < kBucketKpt; ++j) {
        const int64_t i = blk * kBucketChunk + threadIdx.x + kBucketThreads * j;
        kk[j] = i < n ? keys[i] : 0ull;
    }
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int log2_ceil(uint64_t cap)
{
    int lc = 0;
    while ((uint64_t(1) << lc) < cap) ++lc;
    return lc;
}

int seg_log_for(uint64_t cap)
{
    const int lc = log2_ceil(cap);
    return lc < kSegLog ? lc : kSegLog;
}

size_t table_bytes(uint64_t cap) { return align256(sizeof(HashHeader) + cap * (sizeof(uint64_t) + sizeof(int32_t))); }

// scratch of the build at p (256-byte aligned)
SegBuild seg_build_layout_at(char *p, int64_t n, uint64_t cap)
{
    SegBuild b;
    b.seg_log = seg_log_for(cap);
    b.bits = log2_ceil(cap) - b.seg_log;
    b.nseg = int64_t(1) << b.bits;
    b.nblk = n > 0 ? (n + kBucketChunk - 1) / kBucketChunk : 1;
    const size_t nb = align256(static_cast<size_t>(n) * sizeof(uint32_t));
    b.bkeys = reinterpret_cast<uint64_t *>(p);
    p += align256(static_cast<size_t>(n) * sizeof(uint64_t));
    b.idx = reinterpret_cast<uint32_t *>(p);
    p += nb;
    b.ovf = reinterpret_cast<uint32_t *>(p);
    p += nb;
    b.hist = reinterpret_cast<uint32_t *>(p);
    p += align256(static_cast<size_t>(b.nseg * b.nblk) * sizeof(uint32_t));
    b.seg_begin = reinterpret_cast<uint32_t *>(p);
    b.seg_end = b.seg_begin + b.nseg;
    b.seg_tot = b.seg_end + b.nseg;
    b.ovf_count = b.seg_tot + b.nseg;
    return b;
}

// scratch of the build, placed after the table in the caller's workspace
SegBuild seg_build_layout(void *ws, int64_t n, uint64_t cap)
{
    return seg_build_layout_at(static_cast<char *>(ws) + table_bytes(cap), n, cap);
}

size_t seg_build_bytes(int64_t n, uint64_t cap)
{
    const int64_t nn = n < 0 ? 0 : n;
    const int bits = log2_ceil(cap) - seg_log_for(cap);
    const int64_t nseg = int64_t(1) << bits;
    const int64_t nblk = nn > 0 ? (nn + kBucketChunk - 1) / kBucketChunk : 1;
    const size_t nb = align256(static_cast<size_t>(nn) * sizeof(uint32_t));
    return align256(static_cast<size_t>(nn) * sizeof(uint64_t)) + 2 * nb +
           align256(static_cast<size_t>(nseg * nblk) * sizeof(uint32_t)) +
           align256(static_cast<size_t>(3 * nseg + 64) * sizeof(uint32_t));
}

// per chunk of kBucketChunk keys: how many fall in each segment
__global__ __launch_bounds__(kBucketThreads) void k_bucket_count(const uint64_t *__restrict__ keys, int64_t n, uint64_t mask,
                                                      int seg_log, int64_t nseg, int64_t nblk,
                                                      uint32_t *__restrict__ hist, HashHeader *hdr, uint64_t cap,
                                                      uint32_t *ovf_count)
{
    extern __shared__ uint32_t cnt[];
    const int64_t blk = bucket_chunk(nblk);
    if (blk >= nblk) return;
    if (blk == 0 && threadIdx.x == 0) {
        hdr->cap = cap;
        hdr->n = n;
        hdr->err = 0;
        hdr->bad = -1;
        *ovf_count = 0;
    }
    for (int64_t s = threadIdx.x; s < nseg; s += blockDim.x) cnt[s] = 0;
    uint64_t kk[kBucketKpt];
    chunk_keys(keys, n, blk, kk);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBucketKpt; ++j)
        if (blk * kBucketChunk + threadIdx.x + kBucketThreads * j < n) atomicAdd(&cnt[(fnv1a64(kk[j]) & mask) >> seg_log], 1u);
    __syncthreads();
    for (int64_t s = threadIdx.x; s < nseg; s += blockDim.x) hist[s * nblk + blk] = cnt[s];
}

// Per segment (one workgroup each): the exclusive prefix of its per-chunk
// counts, in place, and its total.
__global__ __launch_bounds__(256) void k_bucket_scan_seg(uint32_t *__restrict__ hist, int64_t nblk,
                                                         uint32_t *__restrict__ seg_tot)
{
    __shared__ uint32_t sc[256];
    uint32_t *row = hist + blockIdx.x * nblk;
    const int64_t per = (nblk + 255) / 256;
    const int64_t b0 = threadIdx.x * per, b1 = b0 + per < nblk ? b0 + per : nblk;
    uint32_t sum = 0;
    for (int64_t k = b0; k < b1; ++k) sum += row[k];
    sc[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? sc[threadIdx.x - off] : 0u;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = sc[threadIdx.x] - sum;
    for (int64_t k = b0; k < b1; ++k) {
        const uint32_t t = row[k];
        row[k] = run;
        run += t;
    }
    if (threadIdx.x == 255) seg_tot[blockIdx.x] = sc[255];
}

// Segment bounds from the segment totals (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_bucket_scan_tot(const uint32_t *__restrict__ seg_tot, int64_t nseg,
                                                          uint32_t *__restrict__ seg_begin,
                                                          uint32_t *__restrict__ seg_end)
{
    __shared__ uint32_t sc[1024];
    uint32_t carry = 0;
    for (int64_t base = 0; base < nseg; base += 1024) {
        const int64_t seg = base + threadIdx.x;
        const uint32_t tot = seg < nseg ? seg_tot[seg] : 0u;
        sc[threadIdx.x] = tot;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t v = threadIdx.x >= off ? sc[threadIdx.x - off] : 0u;
            __syncthreads();
            sc[threadIdx.x] += v;
            __syncthreads();
        }
        if (seg < nseg) {
            seg_begin[seg] = carry + sc[threadIdx.x] - tot;
            seg_end[seg] = carry + sc[threadIdx.x];
        }
        carry += sc[1023];
        __syncthreads();
    }
}

// keys and their indices into their segment's range (order inside a segment
// is free).  The keys travel with the indices: the segment build then reads
// both contiguously instead of gathering each key through its index (keys of
// one segment lie about a chunk apart, one cache line per 8-byte key).
__global__ __launch_bounds__(kBucketThreads) void k_bucket_scatter(const uint64_t *__restrict__ keys, int64_t n, uint64_t mask,
                                                        int seg_log, int64_t nseg, int64_t nblk,
                                                        const uint32_t *__restrict__ hist,
                                                        const uint32_t *__restrict__ seg_begin,
                                                        uint64_t *__restrict__ bkeys, uint32_t *__restrict__ idx)
{
    extern __shared__ uint32_t cur[];
    const int64_t blk = bucket_chunk(nblk);
    if (blk >= nblk) return;
    uint64_t kk[kBucketKpt];
    chunk_keys(keys, n, blk, kk);
    for (int64_t s = threadIdx.x; s < nseg; s += blockDim.x) cur[s] = seg_begin[s] + hist[s * nblk + blk];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBucketKpt; ++j) {
        const int64_t i = blk * kBucketChunk + threadIdx.x + kBucketThreads * j;
        if (i < n) {
            const uint32_t pos = atomicAdd(&cur[(fnv1a64(kk[j]) & mask) >> seg_log], 1u);
            bkeys[pos] = kk[j];
            idx[pos] = static_cast<uint32_t>(i);
        }
    }
}

__global__ __launch_bounds__(kSegThreads) void k_seg_build(const uint64_t *__restrict__ bkeys,
                                                   const uint32_t *__restrict__ seg_begin,
                                                   const uint32_t *__restrict__ seg_end,
                                                   const uint32_t *__restrict__ idx, HashHeader *hdr,
                                                   uint64_t *tkeys, int32_t *tvals, uint64_t mask, int seg_log,
                                                   uint32_t *ovf_count, uint32_t *ovf)
{
    __shared__ unsigned long long lk[kSegMax];
    __shared__ int32_t lv[kSegMax];
    const int seg = 1 << seg_log;
    const int64_t s = blockIdx.x;
    for (int j = threadIdx.x; j < seg; j += blockDim.x) {
        lk[j] = 0ull;
        lv[j] = 0;
    }
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(s) << seg_log;
    const uint32_t e_begin = seg_begin[s], e_end = seg_end[s];
    // kSegKpt entries per thread per pass, their keys and indices loaded
    // together, so that a thread waits for memory once per pass rather than
    // once per key (a segment holds about 2048 keys at the table's load
    // factor: one pass)
    for (uint32_t e0 = e_begin; e0 < e_end; e0 += kSegThreads * kSegKpt) {
        uint32_t ii[kSegKpt];
        uint64_t kk[kSegKpt];
        // the loads are unconditional (past the segment's end they repeat its
        // last entry, which exists inside this loop): loads in branches are
        // each waited for before the next one is issued
#pragma unroll
        for (int j = 0; j < kSegKpt; ++j) {
            const uint32_t e = e0 + threadIdx.x + kSegThreads * j;
            const uint32_t ec = e < e_end ? e : e_end - 1;
            ii[j] = idx[ec];
            kk[j] = bkeys[ec];
        }
#pragma unroll
        for (int j = 0; j < kSegKpt; ++j) {
            if (e0 + threadIdx.x + kSegThreads * j >= e_end) continue;
            const uint32_t i = ii[j];
            const uint64_t key = kk[j];
            if (key == 0) {
                flag_error(hdr, RG_EINVAL, i);
                continue;
            }
            int local = static_cast<int>((fnv1a64(key) & mask) - base);
            bool placed = false;
            for (; local < seg; ++local) {
                const unsigned long long prev = atomicCAS(&lk[local], 0ull, static_cast<unsigned long long>(key));
                if (prev == 0ull) {
                    lv[local] = static_cast<int32_t>(i);
                    placed = true;
                    break;
                }
                if (prev == key) {
                    flag_error(hdr, RG_EDUPKEY, i);
                    placed = true;
                    break;
                }
            }
            if (!placed) ovf[atomicAdd(ovf_count, 1u)] = i;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < seg; j += blockDim.x) {
        tkeys[base + j] = lk[j];
        tvals[base + j] = lv[j];
    }
}

// the probe sequences that ran past their segment, on the finished table
__global__ void k_seg_overflow(const uint64_t *__restrict__ keys, const uint32_t *ovf_count,
                               const uint32_t *__restrict__ ovf, HashHeader *hdr, uint64_t *tkeys, int32_t *tvals,
                               uint64_t mask)
{
    const uint32_t m = *ovf_count;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const uint32_t i = ovf[t];
        hash_insert_one(hdr, tkeys, tvals, mask, keys[i], i);
    }
}

__global__ void k_hash_lookup(const uint64_t *__restrict__ keys, const int32_t *__restrict__ vals, uint64_t mask,
                              const uint64_t *__restrict__ q, int64_t m, int32_t *__restrict__ out)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t key = q[i];
    out[i] = key == 0 ? -1 : hash_probe(keys, vals, mask, key);
}

// `list` (optional) maps positions 0..n-1 to oct indices
__global__ __launch_bounds__(256) void k_neighbours(const uint64_t *__restrict__ okeys, const int32_t *__restrict__ list,
                                                    int64_t n, int lmin, int bc, int lmax_zero, HashHeader *hdr,
                                                    const uint64_t *__restrict__ keys, const int32_t *__restrict__ vals,
                                                    uint64_t mask, int32_t *__restrict__ nbr27,
                                                    int32_t *__restrict__ father_cell, uint32_t *__restrict__ son_mask)
{
    __shared__ NbrGroup grp;
    const int64_t first = int64_t(blockIdx.x) * kNbrOcts;
    const int64_t left = n - first;
    const NbrTable tab{okeys, hdr, keys, vals, mask, nbr27, father_cell, son_mask, lmin, bc, lmax_zero};
    nbr_octs_body(tab, list, first, left < kNbrOcts ? static_cast<int>(left) : kNbrOcts, grp);
}

__global__ __launch_bounds__(256) void k_neighbours_brick(const uint64_t *__restrict__ okeys,
                                                          const int32_t *__restrict__ bricks, int64_t nbricks,
                                                          int lmin, int bc, int lmax_zero, HashHeader *hdr,
                                                          const uint64_t *__restrict__ keys,
                                                          const int32_t *__restrict__ vals, uint64_t mask,
                                                          int32_t *__restrict__ nbr27,
                                                          int32_t *__restrict__ father_cell,
                                                          uint32_t *__restrict__ son_mask)
{
    __shared__ NbrBrick nb;
    const int64_t per_xcd = (nbricks + 7) / 8;
    const int64_t b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= nbricks) return;
    const NbrTable tab{okeys, hdr, keys, vals, mask, nbr27, father_cell, son_mask, lmin, bc, lmax_zero};
    nbr_brick_body(tab, bricks[b], nb);
}

}  // namespace

rg_status neighbours_scheduled(void *d_ws, const uint64_t *d_keys, int64_t n, int lmin, int lmax, int64_t n_below_lmax,
                               int bc, const int32_t *bricks, int64_t nbricks, const int32_t *rest, int64_t nrest,
                               int32_t *d_nbr27, int32_t *d_father_cell, uint32_t *d_son_mask, hipStream_t s)
{
    const uint64_t cap = hash_capacity(n);
    HashView h = hash_view(d_ws, cap);
    // only the octs below the finest level can be fathers: their masks are
    // cleared before the children set bits in them; the kernels write the
    // finest level's masks (no children) themselves
    RG_REQUIRE(n_below_lmax >= 0 && n_below_lmax <= n, "bad level range");
    RG_TRY(fill_u32(d_son_mask, n_below_lmax, 0u, s));
    if (nbricks > 0) {
        k_neighbours_brick<<<static_cast<unsigned>(8 * ((nbricks + 7) / 8)), 256, 0, s>>>(
            d_keys, bricks, nbricks, lmin, bc, lmax, h.hdr, h.keys, h.vals, h.mask, d_nbr27, d_father_cell,
            d_son_mask);
        RG_TRY(launch_status("brick neighbours"));
    }
    if (nrest > 0) {
        const int64_t blocks = (nrest + kNbrOcts - 1) / kNbrOcts;
        k_neighbours<<<static_cast<unsigned>(blocks), 256, 0, s>>>(d_keys, rest, nrest, lmin, bc, lmax, h.hdr,
                                                                   h.keys, h.vals, h.mask, d_nbr27, d_father_cell,
                                                                   d_son_mask);
        RG_TRY(launch_status("neighbours"));
    }
    return RG_OK;
}

rg_status fill_u32(uint32_t *d, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return RG_OK;
    k_fill_u32<<<grid_for(n, 256), 256, 0, s>>>(d, n, v);
    return launch_status("fill_u32");
}

rg_status fill_u64(uint64_t *d, int64_t n, uint64_t v, hipStream_t s)
{
    if (n <= 0) return RG_OK;
    k_fill_u64<<<grid_for(n, 256), 256, 0, s>>>(d, n, v);
    return launch_status("fill_u64");
}

namespace {

// Builds the table at d_table (header + slots) from the keys, with the
// build's scratch (bucketing, overflow lists) at b.
rg_status hash_build_into(const uint64_t *d_keys, int64_t n, void *d_table, const SegBuild &b, hipStream_t s)
{
    const uint64_t cap = hash_capacity(n);
    HashView h = hash_view(d_table, cap);
    const size_t cnt_bytes = static_cast<size_t>(b.nseg) * sizeof(uint32_t);
    RG_REQUIRE(cnt_bytes <= 64 * 1024, "table too large for the bucketed build (%lld segments)", (long long)b.nseg);
    k_bucket_count<<<bucket_grid(b.nblk), kBucketThreads, cnt_bytes, s>>>(d_keys, n, h.mask, b.seg_log, b.nseg, b.nblk,
                                                                         b.hist, h.hdr, cap, b.ovf_count);
    RG_TRY(launch_status("rg_hash_build count"));
    k_bucket_scan_seg<<<static_cast<unsigned>(b.nseg), 256, 0, s>>>(b.hist, b.nblk, b.seg_tot);
    RG_TRY(launch_status("rg_hash_build scan"));
    k_bucket_scan_tot<<<1, 1024, 0, s>>>(b.seg_tot, b.nseg, b.seg_begin, b.seg_end);
    RG_TRY(launch_status("rg_hash_build bounds"));
    if (n > 0) {
        k_bucket_scatter<<<bucket_grid(b.nblk), kBucketThreads, cnt_bytes, s>>>(
            d_keys, n, h.mask, b.seg_log, b.nseg, b.nblk, b.hist, b.seg_begin, b.bkeys, b.idx);
        RG_TRY(launch_status("rg_hash_build scatter"));
    }
    const uint32_t *idx = b.idx;
    k_seg_build<<<static_cast<unsigned>(b.nseg), kSegThreads, 0, s>>>(b.bkeys, b.seg_begin, b.seg_end, idx, h.hdr, h.keys,
                                                              h.vals, h.mask, b.seg_log, b.ovf_count, b.ovf);
    RG_TRY(launch_status("rg_hash_build segments"));
    k_seg_overflow<<<64, 256, 0, s>>>(d_keys, b.ovf_count, b.ovf, h.hdr, h.keys, h.vals, h.mask);
    return launch_status("rg_hash_build overflow");
}

// ---------------------------------------------------------------------------
// Scratch of rg_hash_build_noalloc: a file-scope device array, one per
// device (each device that loads the library holds its own copy at its own
// address until the process ends).  Host code never uses the array's name as
// an address: the first call on a device, with that device current, asks
// for the device address with hipGetSymbolAddress and keeps it per device.
// Sized for the largest table the entry point accepts (kNoAllocMaxKeys keys:
// capacity 2^23 slots, 2048 segments of 4096 slots, 1024 chunks of 4096
// keys): the bucketed keys (32 MiB), key-index and overflow lists of 16 MiB
// each, per-chunk counts of 8 MiB, per-segment bounds.  The build writes every word it later reads
// (its first kernel clears the overflow counter), so no call depends on
// what the previous one left; calls that overlap on one device race.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxKeys = int64_t(1) << 22;
constexpr size_t kNoAllocScratchBytes = size_t(kNoAllocMaxKeys) * 8 + 2 * (size_t(kNoAllocMaxKeys) * 4) +
                                        size_t(2048) * 1024 * 4 +
                                        ((size_t(3 * 2048 + 64) * 4 + 255) & ~size_t(255));
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kScratchDevices] = {};

rg_status noalloc_scratch(char *&out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(RG_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kScratchDevices) return fail(RG_ENOTSUP, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail(RG_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    out = g_scratch_ptr[dev];
    return RG_OK;
}

}  // namespace

}  // namespace rg

using namespace rg;

extern "C" {

rg_status rg_encode_keys(const int32_t *d_ijkl, int64_t n, uint64_t *d_keys, void *stream)
{
    RG_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return RG_OK;
    RG_REQUIRE(d_ijkl && d_keys, "null pointer");
    RG_REQUIRE(aligned(d_ijkl, 16) && aligned(d_keys, 8), "misaligned pointer");
    k_encode<<<grid_for(n, 256), 256, 0, as_stream(stream)>>>(d_ijkl, n, d_keys);
    return launch_status("rg_encode_keys");
}

rg_status rg_decode_keys(const uint64_t *d_keys, int64_t n, int32_t *d_ijkl, void *stream)
{
    RG_REQUIRE(n >= 0, "n < 0");
    if (n == 0) return RG_OK;
    RG_REQUIRE(d_ijkl && d_keys, "null pointer");
    RG_REQUIRE(aligned(d_ijkl, 16) && aligned(d_keys, 8), "misaligned pointer");
    k_decode<<<grid_for(n, 256), 256, 0, as_stream(stream)>>>(d_keys, n, d_ijkl);
    return launch_status("rg_decode_keys");
}

size_t rg_sort_workspace_bytes(int64_t n)
{
    if (n <= 0) return 256;
    size_t temp = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, temp, static_cast<const uint64_t *>(nullptr),
                                       static_cast<uint64_t *>(nullptr), static_cast<const int32_t *>(nullptr),
                                       static_cast<int32_t *>(nullptr), static_cast<int>(n));
    size_t iota = (static_cast<size_t>(n) * sizeof(int32_t) + 255) & ~size_t(255);
    return iota + ((temp + 255) & ~size_t(255)) + 256;
}

}  // extern "C"

// radix sort over the low `end_bit` bits (keys of levels <= L fit 3L bits)
rg_status rg::sort_keys_bits(const uint64_t *d_keys_in, int64_t n, uint64_t *d_keys_out, int32_t *d_perm, void *d_ws,
                             size_t ws_bytes, int end_bit, hipStream_t s)
{
    RG_REQUIRE(n >= 0 && n <= INT32_MAX, "n out of range");
    if (n == 0) return RG_OK;
    RG_REQUIRE(d_keys_in && d_keys_out && d_perm && d_ws, "null pointer");
    RG_REQUIRE(d_keys_in != d_keys_out, "in-place sort is not supported");
    RG_REQUIRE(ws_bytes >= rg_sort_workspace_bytes(n), "sort workspace too small");
    RG_REQUIRE(aligned(d_ws, 256), "workspace must be 256-byte aligned");
    RG_REQUIRE(end_bit > 0 && end_bit <= 64, "bad key width");
    int32_t *iota = static_cast<int32_t *>(d_ws);
    size_t iota_bytes = (static_cast<size_t>(n) * sizeof(int32_t) + 255) & ~size_t(255);
    void *temp = static_cast<char *>(d_ws) + iota_bytes;
    size_t temp_bytes = ws_bytes - iota_bytes;
    k_iota<<<grid_for(n, 256), 256, 0, s>>>(iota, n);
    RG_TRY(launch_status("sort iota"));
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, d_keys_in, d_keys_out, iota, d_perm,
                                                      static_cast<int>(n), 0, end_bit, s);
    if (e != hipSuccess) return fail(RG_EHIP, "radix sort: %s", hipGetErrorString(e));
    return launch_status("radix sort");
}

extern "C" {

rg_status rg_sort_keys(const uint64_t *d_keys_in, int64_t n, uint64_t *d_keys_out, int32_t *d_perm, void *d_ws,
                       size_t ws_bytes, void *stream)
{
    return sort_keys_bits(d_keys_in, n, d_keys_out, d_perm, d_ws, ws_bytes, 64, as_stream(stream));
}

rg_status rg_level_ranges(const uint64_t *d_sorted_keys, int64_t n, int64_t *d_level_begin, void *stream)
{
    RG_REQUIRE(n >= 0, "n < 0");
    RG_REQUIRE(d_level_begin, "null pointer");
    hipStream_t s = as_stream(stream);
    if (n == 0) {
        k_zero_i64<<<1, 64, 0, s>>>(d_level_begin, RG_MAX_LEVEL + 2);
        return launch_status("rg_level_ranges");
    }
    RG_REQUIRE(d_sorted_keys, "null pointer");
    k_level_ranges<<<grid_for(n, 256), 256, 0, s>>>(d_sorted_keys, n, d_level_begin);
    return launch_status("rg_level_ranges");
}

rg_status rg_permute_rows(const double *d_in, const int32_t *d_perm, int64_t n_rows, int row_doubles, double *d_out,
                          void *stream)
{
    RG_REQUIRE(n_rows >= 0 && row_doubles > 0, "bad size");
    if (n_rows == 0) return RG_OK;
    RG_REQUIRE(d_in && d_perm && d_out, "null pointer");
    RG_REQUIRE(d_in != d_out, "in-place permutation is not supported");
    k_permute_rows<<<grid_for(n_rows * row_doubles, 256), 256, 0, as_stream(stream)>>>(d_in, d_perm, n_rows,
                                                                                      row_doubles, d_out);
    return launch_status("rg_permute_rows");
}

size_t rg_hash_workspace_bytes(int64_t n_keys)
{
    const int64_t n = n_keys < 0 ? 0 : n_keys;
    const uint64_t cap = hash_capacity(n);
    return table_bytes(cap) + seg_build_bytes(n, cap);
}

uint64_t rg_fnv1a64(uint64_t key) { return fnv1a64(key); }

uint64_t rg_key_host(int32_t i, int32_t j, int32_t k, int32_t l) { return oct_key(i, j, k, l); }

void rg_key_coords_host(uint64_t key, int32_t *h_ijkl)
{
    if (!h_ijkl) return;
    key_coords(key, h_ijkl[0], h_ijkl[1], h_ijkl[2], h_ijkl[3]);
}

rg_status rg_hash_build(const uint64_t *d_keys, int64_t n, void *d_ws, size_t ws_bytes, void *stream)
{
    RG_REQUIRE(n >= 0 && n <= INT32_MAX, "n out of range");
    RG_REQUIRE(d_ws && (n == 0 || d_keys), "null pointer");
    RG_REQUIRE(aligned(d_ws, 256), "workspace must be 256-byte aligned");
    const uint64_t cap = hash_capacity(n);
    if (ws_bytes < rg_hash_workspace_bytes(n))
        return fail(RG_EFULL, "hash workspace holds %zu bytes, %zu needed", ws_bytes, rg_hash_workspace_bytes(n));
    return hash_build_into(d_keys, n, d_ws, seg_build_layout(d_ws, n, cap), as_stream(stream));
}

rg_status rg_hash_build_noalloc(const uint64_t *d_keys, int64_t n, void *d_table, size_t table_bytes_given,
                                void *stream)
{
    RG_REQUIRE(n >= 0 && n <= kNoAllocMaxKeys, "n = %lld: the build without allocation takes at most %lld keys",
               static_cast<long long>(n), static_cast<long long>(kNoAllocMaxKeys));
    RG_REQUIRE(d_table && (n == 0 || d_keys), "null pointer");
    RG_REQUIRE(aligned(d_table, 256), "table must be 256-byte aligned");
    const uint64_t cap = hash_capacity(n);
    if (table_bytes_given < table_bytes(cap))
        return fail(RG_EFULL, "hash table holds %zu bytes, %zu needed", table_bytes_given, table_bytes(cap));
    const size_t need = seg_build_bytes(n, cap);
    RG_REQUIRE(need <= kNoAllocScratchBytes, "build scratch of %zu bytes exceeds the static %zu", need,
               kNoAllocScratchBytes);
    char *scratch_ptr = nullptr;
    RG_TRY(noalloc_scratch(scratch_ptr));
    return hash_build_into(d_keys, n, d_table, seg_build_layout_at(scratch_ptr, n, cap), as_stream(stream));
}

// The capacity is recorded in the header on the device; host callers pass the
// key count they built with, which fixes the capacity the same way.
static rg_status read_capacity(const void *d_ws, uint64_t &cap, hipStream_t s)
{
    HashHeader h;
    hipError_t e = hipMemcpyAsync(&h, d_ws, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(RG_EHIP, "reading hash header: %s", hipGetErrorString(e));
    cap = h.cap;
    return RG_OK;
}

rg_status rg_hash_lookup(const void *d_ws, const uint64_t *d_q, int64_t m, int32_t *d_idx, void *stream)
{
    RG_REQUIRE(m >= 0, "m < 0");
    if (m == 0) return RG_OK;
    RG_REQUIRE(d_ws && d_q && d_idx, "null pointer");
    hipStream_t s = as_stream(stream);
    uint64_t cap = 0;
    RG_TRY(read_capacity(d_ws, cap, s));
    RG_REQUIRE(cap >= 16 && (cap & (cap - 1)) == 0, "workspace holds no built table");
    HashView h = hash_view(const_cast<void *>(d_ws), cap);
    k_hash_lookup<<<grid_for(m, 256), 256, 0, s>>>(h.keys, h.vals, h.mask, d_q, m, d_idx);
    return launch_status("rg_hash_lookup");
}

rg_status rg_check(const void *d_ws, int64_t *h_bad_index, void *stream)
{
    hipStream_t s = as_stream(stream);
    if (!d_ws) return check_sink(h_bad_index, s);
    HashHeader h;
    hipError_t e = hipMemcpyAsync(&h, d_ws, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(RG_EHIP, "rg_check: %s", hipGetErrorString(e));
    if (h_bad_index) *h_bad_index = h.err ? h.bad : -1;
    if (h.err) return fail(static_cast<rg_status>(h.err), "device reported %s at index %lld",
                           rg_status_string(h.err), static_cast<long long>(h.bad));
    return RG_OK;
}

rg_status rg_build_neighbours(void *d_ws, const uint64_t *d_keys, int64_t n, int lmin, int bc, int32_t *d_nbr27,
                              int32_t *d_father_cell, uint32_t *d_son_mask, void *stream)
{
    RG_REQUIRE(n >= 0 && n <= (int64_t(1) << 28), "n out of range");
    if (n == 0) return RG_OK;
    RG_REQUIRE(d_ws && d_keys && d_nbr27 && d_father_cell && d_son_mask, "null pointer");
    RG_REQUIRE(bc == RG_BC_PERIODIC || bc == RG_BC_OUTFLOW, "bad boundary type %d", bc);
    RG_REQUIRE(lmin >= 1 && lmin <= RG_MAX_LEVEL, "bad lmin %d", lmin);
    const uint64_t cap = hash_capacity(n);
    HashView h = hash_view(d_ws, cap);
    hipStream_t s = as_stream(stream);
    RG_TRY(fill_u32(d_son_mask, n, 0u, s));
    const int64_t blocks = (n + kNbrOcts - 1) / kNbrOcts;
    k_neighbours<<<static_cast<unsigned>(blocks), 256, 0, s>>>(d_keys, nullptr, n, lmin, bc, RG_MAX_LEVEL + 1, h.hdr,
                                                               h.keys, h.vals,
                                                               h.mask, d_nbr27, d_father_cell, d_son_mask);
    return launch_status("rg_build_neighbours");
}

}  // extern "C"

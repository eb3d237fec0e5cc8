// rg_internal.hpp -- shared pieces of the gfx950 library behind include/rg.h.
//
// Device helpers for the oct keys (Sec. 2.1 key tuple, Sec. 2.2 Hilbert
// order) and the FNV-1a hash (Sec. 2.1, Sec. 6), the hash workspace header,
// and host-side error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "rg.h"

namespace rg {

// ---------------------------------------------------------------------------
// error plumbing (host)
// ---------------------------------------------------------------------------

void set_detail(const std::string &s);
rg_status fail(rg_status st, const char *fmt, ...);
// checks hipGetLastError() after a launch
rg_status launch_status(const char *what);

#define RG_REQUIRE(cond, ...)                                 \
    do {                                                      \
        if (!(cond)) return ::rg::fail(RG_EINVAL, __VA_ARGS__); \
    } while (0)

#define RG_TRY(expr)                          \
    do {                                      \
        rg_status _st = (expr);               \
        if (_st != RG_OK) return _st;         \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

struct HashHeader;
__device__ inline void flag_error(HashHeader *hdr, int code, int64_t bad);

// Folds a limit m into *p, the bits of a positive double (+inf at first):
// positive doubles order like their bit patterns, so a 64-bit atomic minimum
// gives the exact minimum in any order.  The stored value is read first and
// the atomic skipped when m cannot lower it -- the value only decreases, so a
// stale read is never below it -- which spares one atomic per workgroup on a
// single address.  m = +inf folds nothing.  A negative m marks a non-finite
// state (see nonfinite_limit): the time step becomes 0, which no finite
// state gives and no later fold can raise, and RG_ENONFINITE is recorded in
// hdr (if not null).
__device__ __forceinline__ void fold_min(unsigned long long *p, double m, HashHeader *hdr)
{
    if (m < 0.0) {
        atomicMin(p, 0ull);
        flag_error(hdr, RG_ENONFINITE, -1);
        return;
    }
    if (!(m < __longlong_as_double(0x7ff0000000000000ll))) return;
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(m));
    if (b < *reinterpret_cast<volatile unsigned long long *>(p)) atomicMin(p, b);
}

// Non-finite tracking beside a running minimum of CFL limits: nf starts at
// 0 and takes nf + 0 * (sp + (rho + E)) for every cell, with sp its signal
// speed; it stays 0 while every state is finite and is NaN from the first
// NaN or infinite value on.  (The speed alone is not enough: the density
// and pressure floors turn a NaN density or energy into the floor value.)
__device__ __forceinline__ void track_finite(double &nf, double sp, const double *U)
{
    nf = __builtin_fma(sp + (U[0] + U[4]), 0.0, nf);
}

// The running minimum to reduce: -1 (the non-finite mark of fold_min) when
// the thread met a non-finite speed
__device__ __forceinline__ double nonfinite_limit(double best, double nf) { return nf == nf ? best : -1.0; }

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline unsigned grid_for(int64_t items, int threads)
{
    int64_t g = (items + threads - 1) / threads;
    return static_cast<unsigned>(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// keys: 3-D Hilbert index after Skilling (2004), evaluated at order 20
// ---------------------------------------------------------------------------

constexpr int kHilbertOrder = 20;

// every third bit: bit b of v goes to bit 3b
__host__ __device__ inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// inverse of spread3
__host__ __device__ inline uint32_t gather3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x100f00f00f00f00full;
    x = (x | (x >> 8)) & 0x001f0000ff0000ffull;
    x = (x | (x >> 16)) & 0x001f00000000ffffull;
    x = (x | (x >> 32)) & 0x1fffffull;
    return static_cast<uint32_t>(x);
}

// One bit plane of the axes -> transpose pass: for every axis, reflect the
// low bits of axis 0 when that axis has the plane bit set, otherwise swap
// the low bits of axis 0 and that axis.
__host__ __device__ inline void hilbert_plane(uint32_t &a0, uint32_t &a1, uint32_t &a2, uint32_t q)
{
    const uint32_t low = q - 1;
    if (a0 & q) a0 ^= low;
    if (a1 & q) {
        a0 ^= low;
    } else {
        uint32_t d = (a0 ^ a1) & low;
        a0 ^= d;
        a1 ^= d;
    }
    if (a2 & q) {
        a0 ^= low;
    } else {
        uint32_t d = (a0 ^ a2) & low;
        a0 ^= d;
        a2 ^= d;
    }
}

// index of (x, y, z), 0 <= x, y, z < 2^20, on the order-20 curve
__host__ __device__ inline uint64_t hilbert_index20(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t a0 = x, a1 = y, a2 = z;
#pragma unroll
    for (int b = kHilbertOrder - 1; b >= 1; --b) hilbert_plane(a0, a1, a2, 1u << b);
    // Gray code across the axes, then the parity correction of the top axis
    a1 ^= a0;
    a2 ^= a1;
    uint32_t flip = 0;
#pragma unroll
    for (int b = kHilbertOrder - 1; b >= 1; --b)
        if (a2 & (1u << b)) flip ^= (1u << b) - 1;
    a0 ^= flip;
    a1 ^= flip;
    a2 ^= flip;
    // transposed index: bit b of axis 0 is index bit 3b+2, axis 1 -> 3b+1, axis 2 -> 3b
    return (spread3(a0) << 2) | (spread3(a1) << 1) | spread3(a2);
}

// point of the order-20 curve at index h
__host__ __device__ inline void hilbert_point20(uint64_t h, uint32_t &x, uint32_t &y, uint32_t &z)
{
    uint32_t a0 = gather3(h >> 2), a1 = gather3(h >> 1), a2 = gather3(h);
    // undo the Gray code
    uint32_t t = a2 >> 1;
    a2 ^= a1;
    a1 ^= a0;
    a0 ^= t;
    // undo the plane passes, lowest plane first, axes in reverse order
#pragma unroll
    for (int b = 1; b < kHilbertOrder; ++b) {
        const uint32_t q = 1u << b, low = q - 1;
        if (a2 & q) {
            a0 ^= low;
        } else {
            uint32_t d = (a0 ^ a2) & low;
            a0 ^= d;
            a2 ^= d;
        }
        if (a1 & q) {
            a0 ^= low;
        } else {
            uint32_t d = (a0 ^ a1) & low;
            a0 ^= d;
            a1 ^= d;
        }
        if (a0 & q) a0 ^= low;
    }
    x = a0;
    y = a1;
    z = a2;
}

// Index of (x, y, z), 0 <= x, y, z < 2^nb, on the order-nb curve.  Equal to
// hilbert_index20 of the coordinates shifted left by 20 - nb, shifted right
// by 3 (20 - nb): the bit planes below the shift are zero and every pass on
// them is a no-op, so only the nb planes of the level are run.
__host__ __device__ inline uint64_t hilbert_index_bits(uint32_t x, uint32_t y, uint32_t z, int nb)
{
    uint32_t a0 = x, a1 = y, a2 = z;
    for (int b = nb - 1; b >= 1; --b) hilbert_plane(a0, a1, a2, 1u << b);
    a1 ^= a0;
    a2 ^= a1;
    uint32_t flip = 0;
    for (int b = nb - 1; b >= 1; --b)
        if (a2 & (1u << b)) flip ^= (1u << b) - 1;
    a0 ^= flip;
    a1 ^= flip;
    a2 ^= flip;
    return (spread3(a0) << 2) | (spread3(a1) << 1) | spread3(a2);
}

// inverse of hilbert_index_bits
__host__ __device__ inline void hilbert_point_bits(uint64_t h, int nb, uint32_t &x, uint32_t &y, uint32_t &z)
{
    uint32_t a0 = gather3(h >> 2), a1 = gather3(h >> 1), a2 = gather3(h);
    uint32_t t = a2 >> 1;
    a2 ^= a1;
    a1 ^= a0;
    a0 ^= t;
    for (int b = 1; b < nb; ++b) {
        const uint32_t q = 1u << b, low = q - 1;
        if (a2 & q) {
            a0 ^= low;
        } else {
            uint32_t d = (a0 ^ a2) & low;
            a0 ^= d;
            a2 ^= d;
        }
        if (a1 & q) {
            a0 ^= low;
        } else {
            uint32_t d = (a0 ^ a1) & low;
            a0 ^= d;
            a1 ^= d;
        }
        if (a0 & q) a0 ^= low;
    }
    x = a0;
    y = a1;
    z = a2;
}

// K = 2^(3(l-1)) + H_(l-1)(i,j,k); 0 for coordinates out of range
__host__ __device__ inline uint64_t oct_key(int32_t i, int32_t j, int32_t k, int32_t l)
{
    if (l < 1 || l > RG_MAX_LEVEL) return 0;
    const int b = l - 1;
    const int32_t n = 1 << b;
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return 0;
    const uint64_t h = hilbert_index_bits(static_cast<uint32_t>(i), static_cast<uint32_t>(j),
                                          static_cast<uint32_t>(k), b);
    return (uint64_t(1) << (3 * b)) + h;
}

__host__ __device__ inline int key_level(uint64_t key)
{
#ifdef __HIP_DEVICE_COMPILE__
    int top = 63 - __clzll(static_cast<long long>(key));
#else
    int top = 63 - __builtin_clzll(key);
#endif
    return top / 3 + 1;
}

// (i, j, k, l) of a valid key
__host__ __device__ inline void key_coords(uint64_t key, int32_t &i, int32_t &j, int32_t &k, int32_t &l)
{
    l = key_level(key);
    const int b = l - 1;
    uint32_t x, y, z;
    hilbert_point_bits(key - (uint64_t(1) << (3 * b)), b, x, y, z);
    i = static_cast<int32_t>(x);
    j = static_cast<int32_t>(y);
    k = static_cast<int32_t>(z);
}

// ---------------------------------------------------------------------------
// FNV-1a, 64 bit, over the 8 little-endian bytes of a key
// ---------------------------------------------------------------------------

__host__ __device__ inline uint64_t fnv1a64(uint64_t key)
{
    uint64_t h = 0xcbf29ce484222325ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        h ^= (key >> (8 * b)) & 0xffull;
        h *= 0x100000001b3ull;
    }
    return h;
}

// ---------------------------------------------------------------------------
// hash workspace: header, then keys[cap], then values[cap]
// ---------------------------------------------------------------------------

struct HashHeader {
    uint64_t cap;      // power of two
    int64_t n;         // keys inserted by the last build
    int32_t err;       // first device-side error (rg_status), 0 if none
    int32_t pad;
    int64_t bad;       // offending key index / oct index
    uint64_t reserved[28];
};
static_assert(sizeof(HashHeader) == 256, "hash header is 256 bytes");

inline uint64_t hash_capacity(int64_t n)
{
    uint64_t want = static_cast<uint64_t>(n < 8 ? 8 : n) * 2;
    uint64_t cap = 16;
    while (cap < want) cap <<= 1;
    return cap;
}

struct HashView {
    HashHeader *hdr;
    uint64_t *keys;
    int32_t *vals;
    uint64_t mask;
};

inline HashView hash_view(void *ws, uint64_t cap)
{
    HashView v;
    v.hdr = static_cast<HashHeader *>(ws);
    v.keys = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + sizeof(HashHeader));
    v.vals = reinterpret_cast<int32_t *>(v.keys + cap);
    v.mask = cap - 1;
    return v;
}

__device__ inline void flag_error(HashHeader *hdr, int code, int64_t bad)
{
    if (hdr && atomicCAS(&hdr->err, 0, code) == 0) hdr->bad = bad;
}

// Where device-side errors of a call go: the header of the tree's hash
// workspace inside rg_step, rg_step_subcycled and rg_batch_create (a
// SinkScope names it), else the library's own per-device error word,
// which rg_check(NULL, ...) reads and clears.  Host side.
HashHeader *err_sink();
HashHeader *current_sink();
struct SinkScope {
    explicit SinkScope(void *d_hash_ws);
    ~SinkScope();
    HashHeader *prev;
};

__device__ inline int32_t hash_probe(const uint64_t *keys, const int32_t *vals, uint64_t mask, uint64_t key)
{
    uint64_t s = fnv1a64(key) & mask;
    int32_t found = -1;
    for (uint64_t it = 0; it <= mask; ++it) {
        // the value is read beside the key and taken by a select ahead of the
        // loop's exit test (a return from inside the test would let the
        // compiler move the load behind the comparison): a probe that hits
        // its first slot waits for one memory round trip, not two
        const uint64_t k = keys[s];
        const int32_t v = vals[s];
        found = k == key ? v : found;
        if (k == key || k == 0) break;
        s = (s + 1) & mask;
    }
    return found;
}

// insert key (index i) by linear probing with a 64-bit compare-and-swap;
// errors are flagged in the header
__device__ inline void hash_insert_one(HashHeader *hdr, uint64_t *keys, int32_t *vals, uint64_t mask, uint64_t key,
                                       int64_t i)
{
    if (key == 0) {
        flag_error(hdr, RG_EINVAL, i);
        return;
    }
    uint64_t s = fnv1a64(key) & mask;
    for (uint64_t it = 0; it <= mask; ++it) {
        unsigned long long prev =
            atomicCAS(reinterpret_cast<unsigned long long *>(keys + s), 0ull, static_cast<unsigned long long>(key));
        if (prev == 0ull) {
            vals[s] = static_cast<int32_t>(i);
            return;
        }
        if (prev == key) {
            flag_error(hdr, RG_EDUPKEY, i);
            return;
        }
        s = (s + 1) & mask;
    }
    flag_error(hdr, RG_EFULL, i);
}

// ---------------------------------------------------------------------------
// misc launches shared by several files
// ---------------------------------------------------------------------------

rg_status fill_u32(uint32_t *d, int64_t n, uint32_t v, hipStream_t s);
// lmax: the tree's finest level; n_below_lmax: the octs before it (the ones
// whose son masks are cleared first)
rg_status neighbours_scheduled(void *d_ws, const uint64_t *d_keys, int64_t n, int lmin, int lmax, int64_t n_below_lmax,
                               int bc, const int32_t *bricks, int64_t nbricks, const int32_t *rest, int64_t nrest,
                               int32_t *d_nbr27, int32_t *d_father_cell, uint32_t *d_son_mask, hipStream_t s);
rg_status sort_keys_bits(const uint64_t *d_keys_in, int64_t n, uint64_t *d_keys_out, int32_t *d_perm, void *d_ws,
                         size_t ws_bytes, int end_bit, hipStream_t s);
rg_status fill_u64(uint64_t *d, int64_t n, uint64_t v, hipStream_t s);
// one 64-bit store by a kernel (graph-capture safe, unlike a memset node)
inline rg_status set_u64(uint64_t *d, uint64_t v, hipStream_t s) { return fill_u64(d, 1, v, s); }

}  // namespace rg

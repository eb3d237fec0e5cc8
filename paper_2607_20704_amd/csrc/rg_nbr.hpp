// rg_nbr.hpp -- neighbour-list bodies (one workgroup of 256 threads).
//
// Paper Sec. 2.1: neighbour = hash_get(i-1,j,k,l), father =
// hash_get(i/2,j/2,k/2,l-1); Sec. 2.3: where the neighbour oct does not
// exist the stencil takes a coarse ghost; Sec. 5: a flat 27-entry list per
// oct built from hash lookups.  Shared by the single-tree kernels and the
// batched kernels.
#pragma once

#include "rg_internal.hpp"

namespace rg {
namespace {

// Per-oct build: 27 threads per oct (one per offset), 9 octs per workgroup.
constexpr int kNbrOcts = 9;

struct NbrTable {
    const uint64_t *okeys;     // the tree's sorted keys
    HashHeader *hdr;
    const uint64_t *keys;      // hash slots
    const int32_t *vals;
    uint64_t mask;
    int32_t *nbr27;
    int32_t *father_cell;
    uint32_t *son_mask;
    int lmin, bc;
    // octs on this level have no children: their son masks are written as
    // 0 here rather than cleared beforehand (RG_MAX_LEVEL + 1: none are)
    int lmax_zero;
};

struct NbrGroup {
    int32_t c[kNbrOcts][4];
    int64_t o[kNbrOcts];
};

// octs list[first .. first+count) (or first .. first+count without a list)
__device__ __forceinline__ void nbr_octs_body(const NbrTable &T, const int32_t *__restrict__ list, int64_t first,
                                              int count, NbrGroup &grp)
{
    const int t = threadIdx.x;
    if (t < kNbrOcts && t < count) {
        const int64_t o = list ? int64_t(list[first + t]) : first + t;
        int32_t i, j, k, l;
        key_coords(T.okeys[o], i, j, k, l);
        grp.c[t][0] = i;
        grp.c[t][1] = j;
        grp.c[t][2] = k;
        grp.c[t][3] = l;
        grp.o[t] = o;
    }
    __syncthreads();
    if (t < 27 * kNbrOcts) {
        const int g = t / 27, slot = t - 27 * g;
        if (g < count) {
            const int64_t o = grp.o[g];
            const int32_t i = grp.c[g][0], j = grp.c[g][1], k = grp.c[g][2], l = grp.c[g][3];
            if (slot == 13) {
                T.nbr27[27 * o + 13] = static_cast<int32_t>(o);
                if (l == T.lmax_zero) T.son_mask[o] = 0u;
                if (l > T.lmin) {
                    int32_t f = hash_probe(T.keys, T.vals, T.mask, T.okeys[o] >> 3);
                    if (f < 0) {
                        flag_error(T.hdr, RG_EUNGRADED, o);
                        T.father_cell[o] = -1;
                    } else {
                        const int bit = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
                        T.father_cell[o] = 8 * f + bit;
                        atomicOr(T.son_mask + f, 1u << bit);
                    }
                } else {
                    T.father_cell[o] = -1;
                }
            } else {
                const int dx = slot % 3 - 1, dy = (slot / 3) % 3 - 1, dz = slot / 9 - 1;
                const int32_t N = 1 << (l - 1);
                int32_t ni = i + dx, nj = j + dy, nk = k + dz;
                bool outside = false;
                if (T.bc == RG_BC_PERIODIC) {
                    ni &= N - 1;
                    nj &= N - 1;
                    nk &= N - 1;
                } else if (ni < 0 || nj < 0 || nk < 0 || ni >= N || nj >= N || nk >= N) {
                    outside = true;
                }
                int32_t e = RG_NBR_OUTSIDE;
                if (!outside) {
                    const uint64_t kn = oct_key(ni, nj, nk, l);
                    e = hash_probe(T.keys, T.vals, T.mask, kn);
                    if (e < 0) {
                        int32_t f = (l > 1) ? hash_probe(T.keys, T.vals, T.mask, kn >> 3) : -1;
                        if (f < 0) {
                            flag_error(T.hdr, RG_EUNGRADED, o);
                            e = 0;
                        } else {
                            e = -1 - (8 * f + (ni & 1) + 2 * (nj & 1) + 4 * (nk & 1));
                        }
                    }
                }
                T.nbr27[27 * o + slot] = e;
            }
        }
    }
}

// Neighbour lists of one complete brick (8^3 octs, keys 512 P .. 512 P + 511,
// consecutive in memory).  Inside the brick every neighbour follows from the
// decoded positions.  The 488 oct slots around the brick lie in the 26
// neighbouring brick-sized cubes; a cube whose first and last keys are both
// in the hash table, 511 entries apart, is complete, and its octs are found
// by key offset from its first one -- two lookups per cube instead of one
// per slot.  Slots in other cubes are looked up one by one (with the
// coarse-cell fallback).  Each sibling group's father is looked up once.
// Every child of the brick's fathers lies in the brick, so their son masks
// are complete (all 8 bits) and are stored directly.
struct NbrBrick {
    int32_t slot[10 * 10 * 10];
    int16_t pos[512];         // local position of the k-th oct in key order
    int16_t sbase[512];       // its slot-table index less one in each direction
    int16_t offs[27];         // slot-table offset of each of the 27 list entries
    int32_t father[64];       // father oct of each sibling group
    int32_t cube[27];         // first oct of each neighbouring cube, else -1
    int32_t cube_last[27];    // last oct of each neighbouring cube, else -1
};

__device__ __forceinline__ void nbr_brick_body(const NbrTable &T, int64_t base, NbrBrick &S)
{
    constexpr int BO = 8, HS = 10;
    const int tid = threadIdx.x;
    int32_t i0, j0, k0, l;
    key_coords(T.okeys[base], i0, j0, k0, l);
    i0 &= ~(BO - 1);
    j0 &= ~(BO - 1);
    k0 &= ~(BO - 1);
    for (int k = tid; k < BO * BO * BO; k += 256) {
        int32_t i, j, kk, ll;
        key_coords(T.okeys[base + k], i, j, kk, ll);
        const int p = (i & 7) + BO * (j & 7) + BO * BO * (kk & 7);
        const int sb = (p & 7) + HS * ((p >> 3) & 7) + HS * HS * (p >> 6);
        S.pos[k] = static_cast<int16_t>(p);
        S.sbase[k] = static_cast<int16_t>(sb);
        S.slot[sb + 1 + HS + HS * HS] = static_cast<int32_t>(base + k);
    }
    const int32_t N = 1 << (l - 1);
    // first and last key of each neighbouring cube, looked up on two lanes
    // at once
    if (tid < 54) {
        const int c = tid < 27 ? tid : tid - 27;
        const int dx = c % 3 - 1, dy = (c / 3) % 3 - 1, dz = c / 9 - 1;
        int32_t bi = i0 + BO * dx, bj = j0 + BO * dy, bk = k0 + BO * dz;
        bool inside = true;
        if (T.bc == RG_BC_PERIODIC) {
            bi &= N - 1;
            bj &= N - 1;
            bk &= N - 1;
        } else {
            inside = bi >= 0 && bj >= 0 && bk >= 0 && bi < N && bj < N && bk < N;
        }
        int32_t f = -1;
        if (inside) {
            const uint64_t kb = oct_key(bi, bj, bk, l) & ~uint64_t(BO * BO * BO - 1);
            f = hash_probe(T.keys, T.vals, T.mask, tid < 27 ? kb : kb + (BO * BO * BO - 1));
        }
        if (tid < 27) S.cube[c] = f;
        else S.cube_last[c] = f;
    } else if (tid < 54 + 27) {
        const int e = tid - 54;
        S.offs[e] = static_cast<int16_t>(e % 3 + HS * ((e / 3) % 3) + HS * HS * (e / 9));
    }
    __syncthreads();
    for (int sidx = tid; sidx < HS * HS * HS; sidx += 256) {
        const int sa = sidx % HS - 1, sb = (sidx / HS) % HS - 1, sc = sidx / (HS * HS) - 1;
        if (sa >= 0 && sa < BO && sb >= 0 && sb < BO && sc >= 0 && sc < BO) continue;
        int32_t ni = i0 + sa, nj = j0 + sb, nk = k0 + sc;
        if (T.bc == RG_BC_PERIODIC) {
            ni &= N - 1;
            nj &= N - 1;
            nk &= N - 1;
        } else if (ni < 0 || nj < 0 || nk < 0 || ni >= N || nj >= N || nk >= N) {
            S.slot[sidx] = RG_NBR_OUTSIDE;
            continue;
        }
        const uint64_t kn = oct_key(ni, nj, nk, l);
        const int cube = (sa < 0 ? 0 : (sa >= BO ? 2 : 1)) + 3 * (sb < 0 ? 0 : (sb >= BO ? 2 : 1)) +
                         9 * (sc < 0 ? 0 : (sc >= BO ? 2 : 1));
        // a cube whose first and last keys are 511 entries apart is complete
        const int32_t f0 = S.cube[cube];
        const int32_t first = f0 >= 0 && S.cube_last[cube] == f0 + (BO * BO * BO - 1) ? f0 : -1;
        int32_t e = first >= 0 ? first + static_cast<int32_t>(kn & uint64_t(BO * BO * BO - 1))
                               : hash_probe(T.keys, T.vals, T.mask, kn);
        if (e < 0) {
            const int32_t f = (l > 1) ? hash_probe(T.keys, T.vals, T.mask, kn >> 3) : -1;
            if (f < 0) {
                flag_error(T.hdr, RG_EUNGRADED, base);
                e = 0;
            } else {
                e = -1 - (8 * f + (ni & 1) + 2 * (nj & 1) + 4 * (nk & 1));
            }
        }
        S.slot[sidx] = e;
    }
    if (tid < BO * BO) {
        int32_t f = -1;
        if (l > T.lmin) {
            f = hash_probe(T.keys, T.vals, T.mask, T.okeys[base + 8 * tid] >> 3);
            if (f < 0) flag_error(T.hdr, RG_EUNGRADED, base + 8 * tid);
            else T.son_mask[f] = 0xffu;
        }
        S.father[tid] = f;
    }
    __syncthreads();
    // list entry q = 27 k + e of the brick for q = tid + 256 i: (k, e) is
    // stepped rather than divided out (256 = 9 * 27 + 13), and the entry's
    // slot is its oct's base index plus the offset of e
    static_assert(27 * BO * BO * BO % 256 == 0, "whole passes of the workgroup over the brick's list");
    {
        int k = tid / 27, e = tid - 27 * (tid / 27);
        int32_t *dst = T.nbr27 + 27 * base + tid;
#pragma unroll 6
        for (int i = 0; i < 27 * BO * BO * BO / 256; ++i) {
            __builtin_nontemporal_store(S.slot[S.sbase[k] + S.offs[e]], dst + 256 * i);
            k += 9;
            e += 13;
            if (e >= 27) {
                e -= 27;
                ++k;
            }
        }
    }
    for (int k = tid; k < BO * BO * BO; k += 256) {
        const int p = S.pos[k];
        const int32_t f = S.father[k >> 3];
        T.father_cell[base + k] = f < 0 ? -1 : 8 * f + ((p & 1) + 2 * ((p >> 3) & 1) + 4 * ((p >> 6) & 1));
        if (l == T.lmax_zero) T.son_mask[base + k] = 0u;
    }
}

}  // namespace
}  // namespace rg

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
    int32_t father[64];       // father oct of each sibling group
    int32_t cube[27];         // first oct of each complete neighbouring cube, else -1
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
        S.pos[k] = static_cast<int16_t>(p);
        S.slot[((p & 7) + 1) + HS * (((p >> 3) & 7) + 1) + HS * HS * ((p >> 6) + 1)] = static_cast<int32_t>(base + k);
    }
    const int32_t N = 1 << (l - 1);
    if (tid < 27) {
        const int dx = tid % 3 - 1, dy = (tid / 3) % 3 - 1, dz = tid / 9 - 1;
        int32_t bi = i0 + BO * dx, bj = j0 + BO * dy, bk = k0 + BO * dz;
        bool inside = true;
        if (T.bc == RG_BC_PERIODIC) {
            bi &= N - 1;
            bj &= N - 1;
            bk &= N - 1;
        } else {
            inside = bi >= 0 && bj >= 0 && bk >= 0 && bi < N && bj < N && bk < N;
        }
        int32_t first = -1;
        if (inside) {
            const uint64_t kb = oct_key(bi, bj, bk, l) & ~uint64_t(BO * BO * BO - 1);
            const int32_t f = hash_probe(T.keys, T.vals, T.mask, kb);
            if (f >= 0 && hash_probe(T.keys, T.vals, T.mask, kb + (BO * BO * BO - 1)) == f + (BO * BO * BO - 1))
                first = f;
        }
        S.cube[tid] = first;
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
        const int32_t first = S.cube[cube];
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
    for (int q = tid; q < 27 * BO * BO * BO; q += 256) {
        const int k = q / 27, e = q - 27 * k;
        const int p = S.pos[k];
        const int a = (p & 7) + e % 3, bb = ((p >> 3) & 7) + (e / 3) % 3, c = (p >> 6) + e / 9;
        T.nbr27[27 * base + q] = S.slot[a + HS * bb + HS * HS * c];
    }
    for (int k = tid; k < BO * BO * BO; k += 256) {
        const int p = S.pos[k];
        const int32_t f = S.father[k >> 3];
        T.father_cell[base + k] = f < 0 ? -1 : 8 * f + ((p & 1) + 2 * ((p >> 3) & 1) + 4 * ((p >> 6) & 1));
    }
}

}  // namespace
}  // namespace rg

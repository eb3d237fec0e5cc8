// rg_sib.hpp -- hydro update of one complete sibling group: the 8 octs of
// one father oct, 4x4x4 cells, on one shared tile.
//
// Paper Sec. 3: grouping octs (nsubgrid) lets neighbouring octs share their
// stencil instead of each gathering its own ghost cells.  In a cell-by-cell
// tree the smallest such group that always exists wherever a cell is split
// is the set of its 8 children; outside the 8^3-oct bricks most octs belong
// to complete groups.  A group's tile spans cell offsets -2..5 per axis
// (relative to the group's low corner) and holds 304 cells (the 64 own
// cells, 96 in the face layer, 96 in the outer layer, 48 along the edges)
// against 8 x 80 for eight per-oct tiles; 160 cells are reconstructed (8 x
// 32 per oct) and 240 faces solved (8 x 36).  Each cell of the tile is
// reached through the neighbour list of the sibling whose own 6^3 tile holds
// it, with the same outside and coarse-ghost rules, and every value is
// formed by the same operations as in the per-oct body, so the two give the
// same bits.
#pragma once

#include "rg_oct.hpp"

namespace rg {
namespace {

constexpr int kSibW = 304;   // stencil cells
constexpr int kSibR = 160;   // reconstructed cells: own, then face layer
constexpr int kSibF = 240;   // faces: 3 axes x 5 planes x 16

struct SibTables {
    int8_t wpos[kSibW][3];   // group-relative positions -2..5 (own cells first: x + 4y + 16z)
    int8_t wsib[kSibW];      // sibling (x + 2y + 4z of its place in the group) whose tile holds the cell
    int16_t tile2w[512];     // (x+2) + 8(y+2) + 64(z+2) -> index into wpos, -1 if unused
    // the same, packed so that a thread reads one word per item:
    // stencil cell: (x+2) | (y+2) << 3 | (z+2) << 6 | sibling << 9
    uint32_t wcode[kSibW];
    // reconstructed cell: its neighbours' indices x-, x+, y-, y+, z-, z+
    // (9 bits each), then x+2, y+2, z+2 (3 bits each) from bit 54
    uint64_t rcode[kSibR];
};

constexpr int sib_tile(int x, int y, int z) { return (x + 2) + 8 * (y + 2) + 64 * (z + 2); }

// place 0 or 1 of the sibling whose 6^3 tile (cells -2..3 around its own
// two) covers group position p along one axis
constexpr int sib_place(int p) { return p < 0 ? 0 : (p > 3 ? 1 : p >> 1); }

constexpr void sib_add(SibTables &t, int &n, int x, int y, int z)
{
    t.wpos[n][0] = static_cast<int8_t>(x);
    t.wpos[n][1] = static_cast<int8_t>(y);
    t.wpos[n][2] = static_cast<int8_t>(z);
    t.wsib[n] = static_cast<int8_t>(sib_place(x) + 2 * sib_place(y) + 4 * sib_place(z));
    t.tile2w[sib_tile(x, y, z)] = static_cast<int16_t>(n);
    ++n;
}

constexpr SibTables make_sib_tables()
{
    SibTables t{};
    for (int i = 0; i < 512; ++i) t.tile2w[i] = -1;
    int n = 0;
    for (int z = 0; z < 4; ++z)
        for (int y = 0; y < 4; ++y)
            for (int x = 0; x < 4; ++x) sib_add(t, n, x, y, z);
    // face layer (reconstructed), then outer layer, per axis and side
    for (int layer = 0; layer < 2; ++layer)
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side)
                for (int q = 0; q < 16; ++q) {
                    int p[3] = {0, 0, 0};
                    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
                    p[a] = layer == 0 ? (side ? 4 : -1) : (side ? 5 : -2);
                    p[t1] = q & 3;
                    p[t2] = q >> 2;
                    sib_add(t, n, p[0], p[1], p[2]);
                }
    // edges: two coordinates in {-1, 4}, the third in 0..3
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 16; ++q) {
            int p[3] = {0, 0, 0};
            const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
            p[a] = q & 3;
            p[u] = (q >> 2) & 1 ? 4 : -1;
            p[v] = (q >> 3) & 1 ? 4 : -1;
            sib_add(t, n, p[0], p[1], p[2]);
        }
    for (int i = 0; i < kSibW; ++i)
        t.wcode[i] = static_cast<uint32_t>((t.wpos[i][0] + 2) | (t.wpos[i][1] + 2) << 3 | (t.wpos[i][2] + 2) << 6 |
                                           t.wsib[i] << 9);
    for (int i = 0; i < kSibR; ++i) {
        const int x = t.wpos[i][0], y = t.wpos[i][1], z = t.wpos[i][2];
        const int nb[6] = {t.tile2w[sib_tile(x - 1, y, z)], t.tile2w[sib_tile(x + 1, y, z)],
                           t.tile2w[sib_tile(x, y - 1, z)], t.tile2w[sib_tile(x, y + 1, z)],
                           t.tile2w[sib_tile(x, y, z - 1)], t.tile2w[sib_tile(x, y, z + 1)]};
        uint64_t c = 0;
        for (int k = 0; k < 6; ++k) c |= static_cast<uint64_t>(nb[k]) << (9 * k);
        c |= static_cast<uint64_t>(x + 2) << 54 | static_cast<uint64_t>(y + 2) << 57 | static_cast<uint64_t>(z + 2) << 60;
        t.rcode[i] = c;
    }
    return t;
}

__constant__ SibTables c_sib = make_sib_tables();

// face on axis a between cells c-1 and c (c = 0..4) along a, at (t1, t2) on
// the other two axes in increasing order
__device__ __forceinline__ int sib_face(int a, int c, int t1, int t2) { return 80 * a + 16 * c + t1 + 4 * t2; }

// neighbour-list slot of face side 2 * axis + high
__device__ __forceinline__ int side_slot(int ax, int hi)
{
    const int d = hi ? 1 : -1;
    return nslot(ax == 0 ? d : 0, ax == 1 ? d : 0, ax == 2 ? d : 0);
}

template <typename R> struct SibSmem {
    int64_t oct[8];             // by place in the group
    int32_t nb[8][27];
    // son masks: [0, 8) the siblings; 8 + 4 side + q the neighbour across
    // side (2 axis + high) of the siblings on that face, q = their place
    // along the two other axes (lower axis first)
    uint32_t sm[32];
    double u[64][NV];           // uold, then unew, of the own cells (x + 4y + 16z)
    union {
        R w[NV][kSibW];         // primitive variables of the stencil cells (planes, lds_get)
        double g[kSibF][NV];    // G = F dt/dx per face
    };
    R fs[2][NV][kSibF];         // face states: [0] left of the face, [1] right (planes)
    double red[8];
};

// son mask holding the cell at group position (x, y, z), one coordinate of
// which may lie one cell outside the group
__device__ __forceinline__ uint32_t sib_mask_at(const uint32_t *sm, int x, int y, int z)
{
    if (x < 0) return sm[8 + 0 + (y >> 1) + 2 * (z >> 1)];
    if (x > 3) return sm[8 + 4 + (y >> 1) + 2 * (z >> 1)];
    if (y < 0) return sm[8 + 8 + (x >> 1) + 2 * (z >> 1)];
    if (y > 3) return sm[8 + 12 + (x >> 1) + 2 * (z >> 1)];
    if (z < 0) return sm[8 + 16 + (x >> 1) + 2 * (y >> 1)];
    if (z > 3) return sm[8 + 20 + (x >> 1) + 2 * (y >> 1)];
    return sm[(x >> 1) + 2 * (y >> 1) + 4 * (z >> 1)];
}

template <typename R, int NT, bool GH>
__device__ __forceinline__ void hydro_sib(const LevelArgs &a, const int32_t *__restrict__ father, int64_t first,
                                          SibSmem<R> &S)
{
    const int tid = threadIdx.x;
    const double r = *a.dt / a.dx;
    const double h64 = 0.5 * r;
    const R h = static_cast<R>(h64);
    const R gam = static_cast<R>(a.gamma);
    const double g1d = 1.0 / (a.gamma - 1.0);
    const R g1 = static_cast<R>(g1d);

    // the siblings by place (the father cell's index in its oct), their
    // neighbour lists and son masks; the places of a consistent tree are a
    // permutation, and an inconsistent one still names octs of the group
    if (tid < 8) S.oct[tid] = first + tid;
    __syncthreads();
    if (tid < 8) {
        const int64_t o = first + tid;
        S.oct[father[o] & 7] = o;
    }
    __syncthreads();
    for (int it = tid; it < 8 * 27; it += NT) {
        const int g = it / 27, s = it - 27 * g;
        S.nb[g][s] = a.nbr27[27 * S.oct[g] + s];
    }
    __syncthreads();
    for (int it = tid; it < 32; it += NT) {
        int e;
        if (it < 8) {
            e = static_cast<int>(S.oct[it]);
        } else {
            const int side = (it - 8) >> 2, q = (it - 8) & 3;
            const int ax = side >> 1, hi = side & 1;
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const int sib = (hi << ax) | ((q & 1) << t1) | ((q >> 1) << t2);
            e = S.nb[sib][side_slot(ax, hi)];
        }
        S.sm[it] = e >= 0 ? a.son[e] : 0u;
    }

    // A: gather uold for the stencil cells, primitive variables
    for (int it = tid; it < kSibW; it += NT) {
        const uint32_t code = c_sib.wcode[it];
        const int sib = static_cast<int>(code >> 9);
        int c[3] = {static_cast<int>(code & 7) - 2 - 2 * (sib & 1), static_cast<int>((code >> 3) & 7) - 2 - 2 * ((sib >> 1) & 1),
                    static_cast<int>((code >> 6) & 7) - 2 - 2 * (sib >> 2)};
        int s[3] = {slot_of(c[0]), slot_of(c[1]), slot_of(c[2])};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (s[ax] != 0) {
                const int fs = nslot(ax == 0 ? s[0] : 0, ax == 1 ? s[1] : 0, ax == 2 ? s[2] : 0);
                if (S.nb[sib][fs] == RG_NBR_OUTSIDE) {
                    c[ax] = s[ax] > 0 ? 1 : 0;
                    s[ax] = 0;
                }
            }
        }
        int e = S.nb[sib][nslot(s[0], s[1], s[2])];
        if (e == RG_NBR_OUTSIDE) e = static_cast<int>(S.oct[sib]);
        const int64_t cell = e >= 0 ? 8 * int64_t(e) + ((c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1))
                                    : (-1 - int64_t(e));
        double U[NV], W[NV];
        if (e >= 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v] = a.uold[NV * cell + v];
        } else if constexpr (GH) {
            coarse_ghost(a, cell, c[0] & 1, c[1] & 1, c[2] & 1, U);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v] = a.ucoarse[NV * cell + v];
        }
        prim64(U, a.gamma, W);
#pragma unroll
        for (int v = 0; v < NV; ++v) S.w[v][it] = static_cast<R>(W[v]);
        if (it < 64) {
#pragma unroll
            for (int v = 0; v < NV; ++v) S.u[it][v] = U[v];
        }
    }
    __syncthreads();

    // B: slopes, predictor and face states of the own and face-layer cells
    for (int it = tid; it < kSibR; it += NT) {
        const uint64_t code = c_sib.rcode[it];
        const int x = static_cast<int>((code >> 54) & 7) - 2, y = static_cast<int>((code >> 57) & 7) - 2,
                  z = static_cast<int>((code >> 60) & 7) - 2;
        R dW[3][NV], Wp[NV];
        reconstruct<R>(ld5(S.w, it).v, ld5(S.w, code & 511).v, ld5(S.w, (code >> 9) & 511).v,
                       ld5(S.w, (code >> 18) & 511).v, ld5(S.w, (code >> 27) & 511).v, ld5(S.w, (code >> 36) & 511).v,
                       ld5(S.w, (code >> 45) & 511).v, h, gam, dW, Wp);
        const int p[3] = {x, y, z};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const bool inside_t = p[t1] >= 0 && p[t1] <= 3 && p[t2] >= 0 && p[t2] <= 3;
            if (!inside_t) continue;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int c = side ? p[ax] + 1 : p[ax];
                if (c < 0 || c > 4) continue;
                R st[NV];
                face_state<R>(Wp, dW[ax], side != 0, st);
                lds_put(S.fs[side ? 0 : 1], sib_face(ax, c, p[t1], p[t2]), st);
            }
        }
    }
    __syncthreads();

    // C: HLLC on the 240 faces
    for (int f = tid; f < kSibF; f += NT) {
        const int ax = f / 80, c = (f / 16) % 5, t1 = f & 3, t2 = (f >> 2) & 3;
        R L[NV], Rr[NV];
        lds_get(L, S.fs[0], f);
        lds_get(Rr, S.fs[1], f);
        bool zero = false;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int pa = c - 1 + k;
            const int px0 = ax == 0 ? pa : t1;
            const int px1 = ax == 1 ? pa : (ax == 0 ? t1 : t2);
            const int px2 = ax == 2 ? pa : t2;
            const int bit = (px0 & 1) + 2 * (px1 & 1) + 4 * (px2 & 1);
            zero = zero || ((sib_mask_at(S.sm, px0, px1, px2) >> bit) & 1u);
        }
        double gf[NV];
        face_flux<R>(L, Rr, ax, gam, g1, r, zero, gf);
#pragma unroll
        for (int v = 0; v < NV; ++v) S.g[f][v] = gf[v];
    }
    __syncthreads();

    // D: update, sibling by sibling so that each writes its 40 values in order
    for (int it = tid; it < 8 * 8 * NV; it += NT) {
        const int sib = it / (8 * NV), k = it - 8 * NV * sib;
        const int cidx = k / NV, v = k - NV * cidx;
        const int x = 2 * (sib & 1) + (cidx & 1), y = 2 * ((sib >> 1) & 1) + ((cidx >> 1) & 1),
                  z = 2 * (sib >> 2) + (cidx >> 2);
        const int own = x + 4 * y + 16 * z;
        const double gxm = S.g[sib_face(0, x, y, z)][v], gxp = S.g[sib_face(0, x + 1, y, z)][v];
        const double gym = S.g[sib_face(1, y, x, z)][v], gyp = S.g[sib_face(1, y + 1, x, z)][v];
        const double gzm = S.g[sib_face(2, z, x, y)][v], gzp = S.g[sib_face(2, z + 1, x, y)][v];
        const double un = ((S.u[own][v] + (gxm - gxp)) + (gym - gyp)) + (gzm - gzp);
        a.unew[8 * NV * S.oct[sib] + k] = un;
        S.u[own][v] = un;
    }

    // E: flux owed to coarse neighbours across the group's outer faces;
    // without a buffer there must be none (a coarse neighbour is reported)
    if (!a.corr) {
        for (int it = tid; it < 8 * 6; it += NT) {
            const int sib = it / 6, side = it - 6 * sib;
            const int ax = side >> 1, hi = side & 1;
            if (((sib >> ax) & 1) != hi) continue;
            const int e = S.nb[sib][side_slot(ax, hi)];
            if (e < 0 && e != RG_NBR_OUTSIDE) flag_error(a.hdr, RG_EINVAL, S.oct[sib]);
        }
    } else {
        for (int it = tid; it < 8 * 6 * NV; it += NT) {
            const int sib = it / (6 * NV), k = it - 6 * NV * sib;
            const int side = k / NV, v = k - NV * side;
            const int ax = side >> 1, hi = side & 1;
            if (((sib >> ax) & 1) != hi) continue;
            const int e = S.nb[sib][side_slot(ax, hi)];
            if (!(e < 0 && e != RG_NBR_OUTSIDE)) continue;
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const int b1 = 2 * ((sib >> t1) & 1), b2 = 2 * ((sib >> t2) & 1);
            const int c = hi ? 4 : 0;
            const double sum = (S.g[sib_face(ax, c, b1, b2)][v] + S.g[sib_face(ax, c, b1 + 1, b2)][v]) +
                               (S.g[sib_face(ax, c, b1, b2 + 1)][v] + S.g[sib_face(ax, c, b1 + 1, b2 + 1)][v]);
            const double d = 0.125 * sum;
            const double val = hi ? d : -d;
            double *dst = a.corr + 30 * (S.oct[sib] - a.corr_base) + k;
            *dst = a.corr_mode == 0 ? val : (a.corr_mode == 1 ? 0.0 : *dst) + val;
        }
    }

    // F: fused CFL limit of the new state over the leaf cells that no
    // coarse-fine correction will change (no split face neighbour)
    if (a.dt_next) {
        __syncthreads();
        double best = __longlong_as_double(0x7ff0000000000000ll);
        double nf = 0.0;
        for (int it = tid; it < 64; it += NT) {
            const int x = it & 3, y = (it >> 2) & 3, z = it >> 4;
            const int bit0 = (x & 1) + 2 * (y & 1) + 4 * (z & 1);
            if ((S.sm[(x >> 1) + 2 * (y >> 1) + 4 * (z >> 1)] >> bit0) & 1u) continue;
            bool touch = false;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int d = side ? 1 : -1;
                    const int px = x + (ax == 0 ? d : 0), py = y + (ax == 1 ? d : 0), pz = z + (ax == 2 ? d : 0);
                    const int bit = (px & 1) + 2 * (py & 1) + 4 * (pz & 1);
                    touch = touch || ((sib_mask_at(S.sm, px, py, pz) >> bit) & 1u);
                }
            }
            if (touch) continue;
            double W[NV];
            prim64(S.u[it], a.gamma, W);
            const double cs = sqrt_pos(div_pos(a.gamma * W[4], W[0]));
            const double sp = ((fabs(W[1]) + fabs(W[2])) + fabs(W[3])) + 3.0 * cs;
            const double cd = a.cfl * (a.dx / sp);
            best = cd < best ? cd : best;
            track_finite(nf, sp, S.u[it]);
        }
        best = nonfinite_limit(best, nf);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(best, off, 64);
            best = o < best ? o : best;
        }
        if ((tid & 63) == 0) S.red[tid >> 6] = best;
        __syncthreads();
        if (tid == 0) {
            double m = S.red[0];
            for (int k = 1; k < NT / 64; ++k) m = S.red[k] < m ? S.red[k] : m;
            fold_min(a.dt_next, m, a.hdr);
        }
    }
}

}  // namespace
}  // namespace rg

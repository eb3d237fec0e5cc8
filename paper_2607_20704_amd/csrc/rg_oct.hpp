// rg_oct.hpp -- per-oct hydro update body (one workgroup, G octs of one level).
//
// Paper Sec. 3: each oct is updated from a 6x6x6 stencil of uold (the oct
// and two ghost cells per side): primitive variables, reconstructed face
// states, HLLC fluxes, conservative update into unew.  Shared by the
// single-level kernel and the batched persistent kernel.
#pragma once

#include "rg_internal.hpp"
#include "rg_math.hpp"

namespace rg {
namespace {

// ---------------------------------------------------------------------------
// stencil tables (positions are cell offsets from the oct origin, -2..3)
// ---------------------------------------------------------------------------

struct StencilTables {
    int8_t wpos[80][3];    // cells whose primitive variables are needed
    int8_t rpos[32][3];    // cells that are reconstructed (8 own + 24 face layer)
    int8_t tile2w[216];    // (x+2) + 6(y+2) + 36(z+2) -> index into wpos, -1 if unused
    // packed so that a thread reads one word per item: stencil cell
    // (x+2) | (y+2) << 3 | (z+2) << 6; reconstructed cell: the indices of
    // itself and of its neighbours x-, x+, y-, y+, z-, z+ (7 bits each), then
    // x+2, y+2, z+2 (3 bits each) from bit 49
    uint16_t wcode[80];
    uint64_t rcode[32];
};

constexpr int tile_index(int x, int y, int z) { return (x + 2) + 6 * (y + 2) + 36 * (z + 2); }

constexpr StencilTables make_tables()
{
    StencilTables t{};
    for (int i = 0; i < 216; ++i) t.tile2w[i] = -1;
    int nw = 0, nr = 0;
    // own cells
    for (int c = 0; c < 8; ++c) {
        int p[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        for (int a = 0; a < 3; ++a) {
            t.wpos[nw][a] = static_cast<int8_t>(p[a]);
            t.rpos[nr][a] = static_cast<int8_t>(p[a]);
        }
        t.tile2w[tile_index(p[0], p[1], p[2])] = static_cast<int8_t>(nw);
        ++nw;
        ++nr;
    }
    // face layer (reconstructed) then outer layer, along each axis
    for (int layer = 0; layer < 2; ++layer)
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side)
                for (int q = 0; q < 4; ++q) {
                    int p[3] = {0, 0, 0};
                    int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
                    p[a] = layer == 0 ? (side ? 2 : -1) : (side ? 3 : -2);
                    p[t1] = q & 1;
                    p[t2] = q >> 1;
                    for (int b = 0; b < 3; ++b) t.wpos[nw][b] = static_cast<int8_t>(p[b]);
                    t.tile2w[tile_index(p[0], p[1], p[2])] = static_cast<int8_t>(nw);
                    ++nw;
                    if (layer == 0) {
                        for (int b = 0; b < 3; ++b) t.rpos[nr][b] = static_cast<int8_t>(p[b]);
                        ++nr;
                    }
                }
    // edge cells: two coordinates in {-1, 2}, the third in {0, 1}
    for (int a = 0; a < 3; ++a)        // the axis that stays inside
        for (int q = 0; q < 8; ++q) {
            int p[3] = {0, 0, 0};
            int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
            p[a] = q & 1;
            p[u] = (q >> 1) & 1 ? 2 : -1;
            p[v] = (q >> 2) & 1 ? 2 : -1;
            for (int b = 0; b < 3; ++b) t.wpos[nw][b] = static_cast<int8_t>(p[b]);
            t.tile2w[tile_index(p[0], p[1], p[2])] = static_cast<int8_t>(nw);
            ++nw;
        }
    for (int i = 0; i < 80; ++i)
        t.wcode[i] = static_cast<uint16_t>((t.wpos[i][0] + 2) | (t.wpos[i][1] + 2) << 3 | (t.wpos[i][2] + 2) << 6);
    for (int i = 0; i < 32; ++i) {
        const int x = t.rpos[i][0], y = t.rpos[i][1], z = t.rpos[i][2];
        const int nb[7] = {t.tile2w[tile_index(x, y, z)],     t.tile2w[tile_index(x - 1, y, z)],
                           t.tile2w[tile_index(x + 1, y, z)], t.tile2w[tile_index(x, y - 1, z)],
                           t.tile2w[tile_index(x, y + 1, z)], t.tile2w[tile_index(x, y, z - 1)],
                           t.tile2w[tile_index(x, y, z + 1)]};
        uint64_t c = 0;
        for (int k = 0; k < 7; ++k) c |= static_cast<uint64_t>(nb[k]) << (7 * k);
        c |= static_cast<uint64_t>(x + 2) << 49 | static_cast<uint64_t>(y + 2) << 52 | static_cast<uint64_t>(z + 2) << 55;
        t.rcode[i] = c;
    }
    return t;
}

__constant__ StencilTables c_tab = make_tables();

// face f = 12 a + 4 c + t1 + 2 t2 on axis a between cells c-1 and c along a;
// (t1, t2) are the other two axes in increasing order
__device__ __forceinline__ int face_id(int a, int c, int t1, int t2) { return 12 * a + 4 * c + t1 + 2 * t2; }

__device__ __forceinline__ int nslot(int sx, int sy, int sz) { return (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1); }

__device__ __forceinline__ int slot_of(int x) { return x < 0 ? -1 : (x > 1 ? 1 : 0); }

// ---------------------------------------------------------------------------
// the level kernel
// ---------------------------------------------------------------------------

struct LevelArgs {
    const int32_t *list;  // if set, the octs are list[oct_begin .. oct_end)
    const double *uold;
    const double *ucoarse;   // coarse ghost cells (the coarser level's state; uold itself in a global step)
    double *unew;
    const int32_t *nbr27;
    const uint32_t *son;
    double *corr;
    int64_t corr_base;
    int corr_mode;        // 0: store the owed flux; 1: store 0 + flux; 2: add it (sums over substeps)
    int ghost;            // coarse ghost cells: 0 injection, 1 minmod-limited linear interpolation
    const double *ucoarse2;   // cells two levels down (neighbours of a coarse ghost cell's own coarse cell)
    int64_t oct_begin, oct_end;
    const double *dt;     // device scalar
    double dx;
    double gamma;
    double cfl;
    unsigned long long *dt_next;   // if set: CFL limit of the new state folded in (bits of a positive double)
    HashHeader *hdr;      // device-side errors: non-finite state, fluxes owed to a coarse cell with no buffer
};

// Values of the fine position at sub-cell (sx, sy, sz) of coarse cell C:
// C's own (injection), or with ghost = 1 C's values plus a quarter of each
// minmod slope, toward the position, taken from C's face neighbours (in C's
// oct, in the neighbouring oct, the coarser cell covering it, or C itself
// outside the domain).
__device__ __forceinline__ void coarse_ghost(const LevelArgs &a, int64_t C, int sx, int sy, int sz, double *U)
{
    double uc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uc[v] = a.ucoarse[NV * C + v];
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = uc[v];
    if (!a.ghost) return;
    const int64_t P = C >> 3;
    const int q = static_cast<int>(C & 7);
    const int sub[3] = {sx, sy, sz};
    for (int ax = 0; ax < 3; ++ax) {
        double un[2][NV];
        for (int d = 0; d < 2; ++d) {   // 0: low neighbour, 1: high
            const int qa = (q >> ax) & 1;
            const double *src = a.ucoarse;
            int64_t cell;
            if (qa != d) {
                cell = 8 * P + (q ^ (1 << ax));
            } else {
                const int slot = nslot(ax == 0 ? (d ? 1 : -1) : 0, ax == 1 ? (d ? 1 : -1) : 0, ax == 2 ? (d ? 1 : -1) : 0);
                const int32_t e2 = a.nbr27[27 * P + slot];
                if (e2 == RG_NBR_OUTSIDE) {
                    cell = C;
                } else if (e2 >= 0) {
                    cell = 8 * int64_t(e2) + (q ^ (1 << ax));
                } else {
                    cell = -1 - int64_t(e2);
                    src = a.ucoarse2;
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) un[d][v] = src[NV * cell + v];
        }
        const double qq = sub[ax] ? 0.25 : -0.25;
#pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = U[v] + qq * minmod<double>(uc[v] - un[0][v], un[1][v] - uc[v]);
    }
}

template <typename R, int G> struct Smem {
    int64_t oct[G];
    int32_t nb[G][27];
    uint32_t sm[G][7];          // son masks: own, then sides x-, x+, y-, y+, z-, z+
    double u[G][8][NV];         // uold of the oct's own cells
    // the stencil's primitives are dead once the face states exist (phase
    // B), before the fluxes are written (phase C): one LDS region serves both
    union {
        R w[G][NV][80];         // primitive variables of the stencil cells (planes, lds_get)
        double g[G][36][NV];    // G = F dt/dx per face
    };
    R fs[G][2][NV][36];         // face states: [0] left of the face, [1] right (planes)
    double red[8];              // block minimum of the fused CFL limit (one per wave)
};

// GH: compiled with the interpolating coarse-ghost path (whose registers
// would otherwise lower every launch's occupancy); a.ghost then selects it
template <typename R, int G, int NT, bool GH = false>
__device__ __forceinline__ void hydro_group(const LevelArgs &a, int64_t first, int count, Smem<R, G> &S)
{
    const int tid = threadIdx.x;
    const double r = *a.dt / a.dx;
    const double h64 = 0.5 * r;
    const R h = static_cast<R>(h64);
    const R gam = static_cast<R>(a.gamma);
    const double g1d = 1.0 / (a.gamma - 1.0);
    const R g1 = static_cast<R>(g1d);

    // oct indices, neighbour entries and son masks
    if (tid < G) S.oct[tid] = tid < count ? (a.list ? int64_t(a.list[first + tid]) : first + tid) : 0;
    __syncthreads();
    for (int it = tid; it < G * 27; it += NT) {
        int g = it / 27, s = it - 27 * g;
        S.nb[g][s] = g < count ? a.nbr27[27 * S.oct[g] + s] : 0;
    }
    __syncthreads();
    for (int it = tid; it < G * 7; it += NT) {
        int g = it / 7, k = it - 7 * g;
        uint32_t m = 0;
        if (g < count) {
            int e;
            if (k == 0) {
                e = static_cast<int>(S.oct[g]);
            } else {
                int ax = (k - 1) >> 1, hi = (k - 1) & 1;
                int sx = ax == 0 ? (hi ? 1 : -1) : 0, sy = ax == 1 ? (hi ? 1 : -1) : 0, sz = ax == 2 ? (hi ? 1 : -1) : 0;
                e = S.nb[g][nslot(sx, sy, sz)];
            }
            if (e >= 0) m = a.son[e];
        }
        S.sm[g][k] = m;
    }

    // A: gather uold for the stencil cells, primitive variables
    for (int it = tid; it < G * 80; it += NT) {
        int g = it / 80, wc = it - 80 * g;
        if (g >= count) continue;
        const int code = c_tab.wcode[wc];
        int c[3] = {(code & 7) - 2, ((code >> 3) & 7) - 2, ((code >> 6) & 7) - 2};
        int s[3] = {slot_of(c[0]), slot_of(c[1]), slot_of(c[2])};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (s[ax] != 0) {
                int fs = nslot(ax == 0 ? s[0] : 0, ax == 1 ? s[1] : 0, ax == 2 ? s[2] : 0);
                if (S.nb[g][fs] == RG_NBR_OUTSIDE) {
                    c[ax] = s[ax] > 0 ? 1 : 0;
                    s[ax] = 0;
                }
            }
        }
        int e = S.nb[g][nslot(s[0], s[1], s[2])];
        // a consistent list never leaves an outside slot here; an
        // inconsistent one reads the oct itself rather than stray memory
        if (e == RG_NBR_OUTSIDE) e = static_cast<int>(S.oct[g]);
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
        for (int v = 0; v < NV; ++v) S.w[g][v][wc] = static_cast<R>(W[v]);
        if (wc < 8) {
#pragma unroll
            for (int v = 0; v < NV; ++v) S.u[g][wc][v] = U[v];
        }
    }
    __syncthreads();

    // B: slopes, predictor and face states
    for (int it = tid; it < G * 32; it += NT) {
        int g = it / 32, rc = it - 32 * g;
        if (g >= count) continue;
        const uint64_t code = c_tab.rcode[rc];
        const int x = static_cast<int>((code >> 49) & 7) - 2, y = static_cast<int>((code >> 52) & 7) - 2,
                  z = static_cast<int>((code >> 55) & 7) - 2;
        R dW[3][NV], Wp[NV];
        reconstruct<R>(ld5(S.w[g], code & 127).v, ld5(S.w[g], (code >> 7) & 127).v, ld5(S.w[g], (code >> 14) & 127).v,
                       ld5(S.w[g], (code >> 21) & 127).v, ld5(S.w[g], (code >> 28) & 127).v,
                       ld5(S.w[g], (code >> 35) & 127).v, ld5(S.w[g], (code >> 42) & 127).v, h,
                       gam, dW, Wp);
        const int p[3] = {x, y, z};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const bool inside_t = p[t1] >= 0 && p[t1] <= 1 && p[t2] >= 0 && p[t2] <= 1;
            if (!inside_t) continue;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                // high-side state sits left of face c = p+1; low-side state right of face c = p
                const int c = side ? p[ax] + 1 : p[ax];
                if (c < 0 || c > 2) continue;
                R st[NV];
                face_state<R>(Wp, dW[ax], side != 0, st);
                lds_put(S.fs[g][side ? 0 : 1], face_id(ax, c, p[t1], p[t2]), st);
            }
        }
    }
    __syncthreads();

    // C: HLLC on the 36 faces
    for (int it = tid; it < G * 36; it += NT) {
        int g = it / 36, f = it - 36 * g;
        if (g >= count) continue;
        const int ax = f / 12, c = (f / 4) % 3, t1 = f & 1, t2 = (f >> 1) & 1;
        R L[NV], Rr[NV];
        lds_get(L, S.fs[g][0], f);
        lds_get(Rr, S.fs[g][1], f);
        // split test for the two cells: position c-1 and c along the axis
        bool zero = false;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int pa = c - 1 + k;
            // cell position (pa along the axis, t1 / t2 across it) without a
            // run-time-indexed array, which would live in scratch memory
            const int px0 = ax == 0 ? pa : t1;
            const int px1 = ax == 1 ? pa : (ax == 0 ? t1 : t2);
            const int px2 = ax == 2 ? pa : t2;
            const int bit = (px0 & 1) + 2 * (px1 & 1) + 4 * (px2 & 1);
            const uint32_t m = pa < 0 ? S.sm[g][1 + 2 * ax] : (pa > 1 ? S.sm[g][2 + 2 * ax] : S.sm[g][0]);
            zero = zero || ((m >> bit) & 1u);
        }
        double gf[NV];
        face_flux<R>(L, Rr, ax, gam, g1, r, zero, gf);
#pragma unroll
        for (int v = 0; v < NV; ++v) S.g[g][f][v] = gf[v];
    }
    __syncthreads();

    // D: update
    for (int it = tid; it < G * 8 * NV; it += NT) {
        int g = it / (8 * NV), k = it - 8 * NV * g;
        if (g >= count) continue;
        const int cidx = k / NV, v = k - NV * cidx;
        const int ix = cidx & 1, iy = (cidx >> 1) & 1, iz = cidx >> 2;
        const double gxm = S.g[g][face_id(0, ix, iy, iz)][v], gxp = S.g[g][face_id(0, ix + 1, iy, iz)][v];
        const double gym = S.g[g][face_id(1, iy, ix, iz)][v], gyp = S.g[g][face_id(1, iy + 1, ix, iz)][v];
        const double gzm = S.g[g][face_id(2, iz, ix, iy)][v], gzp = S.g[g][face_id(2, iz + 1, ix, iy)][v];
        const double un = ((S.u[g][cidx][v] + (gxm - gxp)) + (gym - gyp)) + (gzm - gzp);
        a.unew[8 * NV * S.oct[g] + k] = un;
        S.u[g][cidx][v] = un;
    }

    // E: flux owed to coarse neighbours.  Without a buffer there must be
    // none: a coarse face neighbour is then reported (its flux is lost).
    if (!a.corr) {
        for (int it = tid; it < G * 6; it += NT) {
            const int g = it / 6, side = it - 6 * g;
            if (g >= count) continue;
            const int ax = side >> 1, hi = side & 1;
            const int e = S.nb[g][nslot(ax == 0 ? (hi ? 1 : -1) : 0, ax == 1 ? (hi ? 1 : -1) : 0,
                                        ax == 2 ? (hi ? 1 : -1) : 0)];
            if (e < 0 && e != RG_NBR_OUTSIDE) flag_error(a.hdr, RG_EINVAL, S.oct[g]);
        }
    } else {
        for (int it = tid; it < G * 6 * NV; it += NT) {
            int g = it / (6 * NV), k = it - 6 * NV * g;
            if (g >= count) continue;
            const int side = k / NV, v = k - NV * side;
            const int ax = side >> 1, hi = side & 1;
            const int e = S.nb[g][nslot(ax == 0 ? (hi ? 1 : -1) : 0, ax == 1 ? (hi ? 1 : -1) : 0,
                                        ax == 2 ? (hi ? 1 : -1) : 0)];
            if (!(e < 0 && e != RG_NBR_OUTSIDE)) continue;
            const int c = hi ? 2 : 0;
            const double sum = (S.g[g][face_id(ax, c, 0, 0)][v] + S.g[g][face_id(ax, c, 1, 0)][v]) +
                               (S.g[g][face_id(ax, c, 0, 1)][v] + S.g[g][face_id(ax, c, 1, 1)][v]);
            const double d = 0.125 * sum;
            const double val = hi ? d : -d;
            double *dst = a.corr + 30 * (S.oct[g] - a.corr_base) + k;
            *dst = a.corr_mode == 0 ? val : (a.corr_mode == 1 ? 0.0 : *dst) + val;
        }
    }

    // F: fused CFL limit of the new state over the group's leaf cells that
    // no coarse-fine correction will change (no split face neighbour)
    if (a.dt_next) {
        __syncthreads();
        double best = __longlong_as_double(0x7ff0000000000000ll);
        double nf = 0.0;
        for (int it = tid; it < G * 8; it += NT) {
            const int g = it >> 3, cidx = it & 7;
            if (g >= count) continue;
            if ((S.sm[g][0] >> cidx) & 1u) continue;
            const int p[3] = {cidx & 1, (cidx >> 1) & 1, cidx >> 2};
            bool touch = false;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    int px[3] = {p[0], p[1], p[2]};
                    px[ax] += side ? 1 : -1;
                    const int bit = (px[0] & 1) + 2 * (px[1] & 1) + 4 * (px[2] & 1);
                    const uint32_t m = px[ax] < 0 ? S.sm[g][1 + 2 * ax] : (px[ax] > 1 ? S.sm[g][2 + 2 * ax] : S.sm[g][0]);
                    touch = touch || ((m >> bit) & 1u);
                }
            }
            if (touch) continue;
            double W[NV];
            prim64(S.u[g][cidx], a.gamma, W);
            const double cs = sqrt_pos(div_pos(a.gamma * W[4], W[0]));
            const double sp = ((fabs(W[1]) + fabs(W[2])) + fabs(W[3])) + 3.0 * cs;
            const double cd = a.cfl * (a.dx / sp);
            best = cd < best ? cd : best;
            track_finite(nf, sp, S.u[g][cidx]);
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

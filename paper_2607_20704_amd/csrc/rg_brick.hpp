// rg_brick.hpp -- plane-sweep hydro update of one complete 8x8x8-oct brick.
//
// Paper Sec. 3 (rock/paper kernels): larger blocks of octs share their
// stencil; the "paper" kernel sweeps a planar stencil through the block.
// Shared by the single-level brick kernel and the batched persistent kernel.
#pragma once

#include "rg_internal.hpp"
#include "rg_math.hpp"

namespace rg {
namespace {

constexpr int BO = 8;          // octs per brick side
constexpr int BC = 16;         // cells per brick side
constexpr int BT = 256;        // threads per workgroup
constexpr int PW = BC + 4;     // plane width with two ghost cells per side
constexpr int HS = BO + 2;     // slot table side: octs -1..8

struct BrickArgs {
    const double *uold;
    double *unew;
    const int32_t *nbr27;
    const uint32_t *son;
    const uint64_t *keys;
    const int32_t *bricks;     // first oct of each brick
    int64_t nbricks;
    const double *dt;
    double dx;
    double gamma;
    int outflow;               // clamp positions outside the domain (zero gradient)
    double cfl;
    unsigned long long *dt_next;   // if set: CFL limit of the new state folded in (bits of a positive double)
    HashHeader *hdr;               // device-side errors (non-finite state)
};

// LDS holds every 5-variable quantity as five planes, one per variable
// (structure of arrays), so that the 64 lanes of a wave, which own
// consecutive cells of a row, read and write consecutive 8-byte words:
// with 40-byte cell records (array of structures) lane i's word sits 10
// dwords after lane i-1's and the accesses of a wave collide in the banks.
constexpr int FXN = BC * (BC + 1);   // x faces: row y, face x (x = 0..16 -> faces -1|0 .. 15|16)
constexpr int FYN = (BC + 1) * BC;   // y faces: face y (y = 0..16), column x

// Face states, written by the reconstruction; each is read by exactly one
// thread in the flux pass, which then overwrites it with the flux of that
// face, so states and fluxes share the storage without a barrier.
//   fx[v][y * (BC + 1) + x]: face (x-1 | x) of row y: the x+ state of cell
//     x-1, then the face's flux;
//   fy[v][y * BC + x]: face (y-1 | y) of column x: the y+ state of cell y-1,
//     then the flux;
//   sxm_hi[v][y], sym_hi[v][x]: the x- / y- states of the ghost cells x = 16
//     (row y) and y = 16 (column x).
template <typename R> struct BrickFaces {
    R fx[NV][FXN];
    R fy[NV][FYN];
    R sxm_hi[NV][BC];
    R sym_hi[NV][BC];
};
static_assert(sizeof(BrickFaces<double>) == sizeof(double) * NV * (FXN + FYN + 2 * BC), "packed face planes");

// The face state that ghost-ring lane (side q, position k) writes: q = 0 the
// x+ state of cell x = -1 in row k (fx, face 0), 1 the x- state of ghost
// x = 16 (sxm_hi), 2 the y+ state of cell y = -1 in column k (fy, face 0),
// 3 the y- state of ghost y = 16 (sym_hi).  Element v sits at flat index
// base + v * stride of the buffer, computed with plain arithmetic: a pointer
// chosen per lane through branches (one pointer per side) was compiled
// wrongly once (the lanes of the last side stored through the pointer of
// the third).
template <typename R> __device__ __forceinline__ void ring_put(BrickFaces<R> &F, int q, int k, const R *src)
{
    const int hi = q & 1, ax = q >> 1;
    const int base = (1 - hi) * ((1 - ax) * (BC + 1) * k + ax * (NV * FXN + k)) +
                     hi * (NV * (FXN + FYN) + ax * NV * BC + k);
    const int stride = (1 - hi) * FXN + hi * BC;
    R *flat = &F.fx[0][0];
#pragma unroll
    for (int v = 0; v < NV; ++v) flat[base + v * stride] = src[v];
}

// NB = 2: two face buffers and two split-flag planes (planes of even and odd
// z), which saves one barrier per plane (see brick_body) for 23 KB more LDS
// in FP64 -- free at two workgroups per CU, which the FP64 kernel's registers
// allow anyway; NB = 1 for variants that fit more workgroups.
// NZ = 2: two bricks stacked along z swept as one column of 32 planes (the
// slot table then spans octs -1..16 in z).
template <typename R, int NB = 1, int NZ = 1> struct BrickSmem {
    BrickFaces<R> u_[NB];           // face states and fluxes (NB = 2: planes of even / odd z)
    int32_t slot[HS * HS * (BO * NZ + 2)];   // oct slots -1..8 (z: -1..8 NZ) around the brick(s): oct
                                             // index inside, neighbour entry outside
    uint8_t son[HS * HS * (BO * NZ + 2)];    // son mask of same-level slot octs, 0 otherwise
    R w[NV][PW * PW];               // primitive variables of the current plane
    R hw[3][NV][4 * BC];            // primitive variables of the reconstructed ghost ring, planes r-1, r, r+1
    uint8_t split[NB][PW * PW];     // split flags of the current plane's cells
    double red[8];                  // block minimum of the fused CFL limit, one per wave
    int32_t any_son;                // some slot oct in reach has a split cell
    // mixed form with one buffer: each column's partial update of the
    // previous plane (its own slot, no sharing), kept here rather than in
    // registers
    double acc[NV][(sizeof(R) == 4 && NB == 1) ? BT : 1];
};

struct Geom {
    int cx0, cy0, cz0;   // global cell coordinates of the brick origin
    int ncell;           // cells per side of the level
    int outflow;
};

// slot index of the oct slot (sa, sb, sc) in [-1, 8]^3
__device__ __forceinline__ int slot_index(int sa, int sb, int sc) { return (sa + 1) + HS * (sb + 1) + HS * HS * (sc + 1); }

// Source of the cell at brick-relative position (x, y, z): its global cell
// id, and whether it is a split cell.  Outside the domain (outflow) the
// position takes the nearest cell inside (zero gradient) and counts as not
// split; a missing same-level oct gives its coarse cell (injection).  GEN =
// false: the brick has no split cell in reach and no position outside the
// domain (checked once per brick), so neither is looked at.
template <bool GEN, typename SM>
__device__ __forceinline__ int64_t source_cell(const SM &S, const Geom &g, int x, int y, int z, bool &split)
{
    bool clamped = false;
    if (GEN && g.outflow) {
        const int gx = g.cx0 + x, gy = g.cy0 + y, gz = g.cz0 + z;
        if (gx < 0) { x = -g.cx0; clamped = true; }
        if (gx >= g.ncell) { x = g.ncell - 1 - g.cx0; clamped = true; }
        if (gy < 0) { y = -g.cy0; clamped = true; }
        if (gy >= g.ncell) { y = g.ncell - 1 - g.cy0; clamped = true; }
        if (gz < 0) { z = -g.cz0; clamped = true; }
        if (gz >= g.ncell) { z = g.ncell - 1 - g.cz0; clamped = true; }
    }
    const int bit = (x & 1) + 2 * (y & 1) + 4 * (z & 1);
    const int si = slot_index(x >> 1, y >> 1, z >> 1);
    int32_t e = S.slot[si];
    split = GEN && !clamped && ((S.son[si] >> bit) & 1u);
    if (e == RG_NBR_OUTSIDE) e = S.slot[slot_index(0, 0, 0)];   // unreachable for a consistent list
    return e >= 0 ? 8 * int64_t(e) + bit : (-1 - int64_t(e));
}

__device__ __forceinline__ void load_u(const double *__restrict__ u, int64_t cell, double *U)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = u[NV * cell + v];
}

// primitive variables in R; returns 1 / rho in double
template <typename R> __device__ __forceinline__ double to_prim(const double *U, double gamma, R *W)
{
    double w[NV];
    const double inv = prim64(U, gamma, w);
#pragma unroll
    for (int v = 0; v < NV; ++v) W[v] = static_cast<R>(w[v]);
    return inv;
}

template <typename R> __device__ __forceinline__ void copy5(R *d, const R *s)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = s[v];
}

// position of the secondary (ghost ring) role of a thread:
//   kind 1: face layer (x = -1 or 16, or y = -1 or 16), reconstructed
//   kind 2: outer ring (x = -2 or 17, or y = -2 or 17)
//   kind 3: inner corners (-1,-1), (16,-1), (-1,16), (16,16)
__device__ __forceinline__ void ring_pos(int kind, int lane, int &x, int &y)
{
    const int q = lane >> 4, k = lane & 15;
    if (kind == 3) {
        x = (lane & 1) ? BC : -1;
        y = (lane & 2) ? BC : -1;
        return;
    }
    const int lo = kind == 1 ? -1 : -2, hi = kind == 1 ? BC : BC + 1;
    if (q == 0) { x = lo; y = k; }
    else if (q == 1) { x = hi; y = k; }
    else if (q == 2) { x = k; y = lo; }
    else { x = k; y = hi; }
}

// Face fluxes in the LDS buffer: the mixed form keeps F in float; FP64
// stores G = F dt/dx once per face (the same product both cells would form)
template <typename R, int N>
__device__ __forceinline__ void store_flux(R (&a)[NV][N], int i, const R *F, double r)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v][i] = sizeof(R) == 8 ? static_cast<R>(static_cast<double>(F[v]) * r) : F[v];
}

template <typename R> __device__ __forceinline__ double flux_G(R f, double r)
{
    return sizeof(R) == 8 ? static_cast<double>(f) : static_cast<double>(f) * r;
}

// hllc flux of one face, zeroed when it touches a split cell (GEN only)
template <bool GEN, typename R>
__device__ __forceinline__ void face_F(const R *L, const R *Rt, int dir, R gamma, R g1, bool zero, R *F)
{
    hllc<R>(L, Rt, dir, gamma, g1, F);
    if constexpr (GEN) {
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = zero ? R(0) : F[v];
    }
}

// G = F dt/dx of the z face, zeroed when it touches a split cell (GEN only)
template <bool GEN, typename R>
__device__ __forceinline__ void face_G(const R *L, const R *Rt, R gamma, R g1, double r, bool zero, double *G)
{
    R F[NV];
    hllc<R>(L, Rt, 2, gamma, g1, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) G[v] = (GEN && zero) ? 0.0 : static_cast<double>(F[v]) * r;
}

// signal speed |u| + |v| + |w| + 3c of a new conserved state, for the CFL
// limit cfl dx / speed
__device__ __forceinline__ double signal_speed(const double *U, double gamma)
{
    double Wn[NV];
    prim64(U, gamma, Wn);
    const double cs = sqrt_pos(div_pos(gamma * Wn[4], Wn[0]));
    return ((fabs(Wn[1]) + fabs(Wn[2])) + fabs(Wn[3])) + 3.0 * cs;
}

// One brick (first oct `base`) by one workgroup of BT threads, each owning
// an interior column.  The ghost ring (loads of the two-cell halo,
// reconstruction of the face layer x = -1, 16 / y = -1, 16, the fluxes of
// the faces x = 16 / y = 16) is shared out to whole waves, with the roles
// rotated by the brick index b so that the extra work lands on a different
// SIMD from brick to brick.  (A fifth wave holding the whole ring measured
// slower: the column waves wait for it at every barrier.)
//
// KU: keep each column's conserved state of the current plane in registers
// until the update instead of reading it again (10 more registers, one
// 40-byte read per cell less).
//
// GEN: the brick has a split cell within reach of its stencil, or an
// outflow wall within two cells; otherwise (GEN = false, decided once per
// brick) the sweep skips the split flags, the zeroed fluxes, the leaf tests
// of the folded time step and the clamping at walls.  Both give the same
// bits where both apply.
template <typename R, bool KU, int NB, bool GEN, int NZ>
__device__ __forceinline__ void brick_sweep(const BrickArgs &a, int64_t b, const Geom &g, BrickSmem<R, NB, NZ> &S);

// Slot table and geometry of the brick whose first oct is `base` (NZ = 2:
// and of the brick directly above it, first oct `base2`), built by NT
// threads; returns GEN (see brick_sweep) for the brick(s).
template <int NT, int NZ, typename SM>
__device__ __forceinline__ bool brick_setup(const BrickArgs &a, int64_t base, int64_t base2, SM &S, Geom &g)
{
    constexpr int ZO = BO * NZ;   // octs along z
    const int tid = threadIdx.x;
    for (int k = tid; k < NZ * BO * BO * BO; k += NT) {
        const bool upper = k >= BO * BO * BO;
        const int64_t o = upper ? base2 + (k - BO * BO * BO) : base + k;
        int32_t i, j, kk, l;
        key_coords(a.keys[o], i, j, kk, l);
        S.slot[slot_index(i & 7, j & 7, (kk & 7) + (upper ? BO : 0))] = static_cast<int32_t>(o);
    }
    if (tid == 0) S.any_son = 0;
    {
        int32_t i, j, kk, l;
        key_coords(a.keys[base], i, j, kk, l);
        g.cx0 = 2 * (i & ~7);
        g.cy0 = 2 * (j & ~7);
        g.cz0 = 2 * (kk & ~7);
        g.ncell = 1 << l;
        g.outflow = a.outflow;
    }
    __syncthreads();
    for (int s = tid; s < HS * HS * (ZO + 2); s += NT) {
        const int sa = s % HS - 1, sb = (s / HS) % HS - 1, sc = s / (HS * HS) - 1;
        const int out = (sa < 0 || sa >= BO) + (sb < 0 || sb >= BO) + (sc < 0 || sc >= ZO);
        int32_t e = RG_NBR_OUTSIDE;
        if (out == 0) {
            e = S.slot[s];
        } else if (out <= 2) {
            // the nearest brick oct and its neighbour entry towards this slot
            const int ca = sa < 0 ? 0 : (sa >= BO ? BO - 1 : sa);
            const int cb = sb < 0 ? 0 : (sb >= BO ? BO - 1 : sb);
            const int cc = sc < 0 ? 0 : (sc >= ZO ? ZO - 1 : sc);
            const int32_t o = S.slot[slot_index(ca, cb, cc)];
            e = a.nbr27[27 * int64_t(o) + (sa - ca + 1) + 3 * (sb - cb + 1) + 9 * (sc - cc + 1)];
        }
        const uint8_t m = e >= 0 ? static_cast<uint8_t>(a.son[e]) : 0;
        S.son[s] = m;
        if (m) S.any_son = 1;
        if (out) S.slot[s] = e;
    }
    __syncthreads();
    const bool wall = g.outflow && (g.cx0 == 0 || g.cy0 == 0 || g.cz0 == 0 || g.cx0 + BC == g.ncell ||
                                    g.cy0 + BC == g.ncell || g.cz0 + NZ * BC == g.ncell);
    return S.any_son != 0 || wall;
}

template <typename R, bool KU = false, int NB = 1, int NZ = 1>
__device__ __forceinline__ void brick_body(const BrickArgs &a, int64_t base, int64_t b, BrickSmem<R, NB, NZ> &S,
                                           int64_t base2 = -1)
{
    Geom g;
    if (brick_setup<BT, NZ>(a, base, base2, S, g))
        brick_sweep<R, KU, NB, true, NZ>(a, b, g, S);
    else
        brick_sweep<R, KU, NB, false, NZ>(a, b, g, S);
}

template <typename R, bool KU, int NB, bool GEN, int NZ>
__device__ __forceinline__ void brick_sweep(const BrickArgs &a, int64_t b, const Geom &g, BrickSmem<R, NB, NZ> &S)
{
    constexpr int ZC = NZ * BC;   // planes swept
    const int tid = threadIdx.x;
    const double r = *a.dt / a.dx;
    const R h = static_cast<R>(0.5 * r);
    const R gam = static_cast<R>(a.gamma);
    const R g1 = static_cast<R>(1.0 / (a.gamma - 1.0));

    // ---- roles
    const int x = tid & 15, y = tid >> 4;
    const int wave = tid >> 6, lane = tid & 63;
    const int ew = static_cast<int>(b & 3);         // wave holding the reconstructed ghost ring this brick
    const bool do_face = wave == ew;
    const bool do_outer = wave == ((ew + 1) & 3);
    const bool do_corner = wave == ((ew + 2) & 3) && lane < 4;
    // faces x = 16 (lanes 0-15) and y = 16 (lanes 16-31), one Riemann pass,
    // on the wave without a ghost-ring role
    const bool extra_faces = wave == ((ew + 3) & 3) && lane < 2 * BC;
    int hx = 0, hy = 0;
    ring_pos(1, lane, hx, hy);      // face layer position of this lane
    const int hq = lane >> 4, hk = lane & 15;

    // own column: primitive variables of planes r-1, r, r+1 and conserved
    // variables of planes r (update) and r+1 (next primitives); secondary
    // position: the conserved variables it needs next
    R Wm[NV], W0[NV], Wp[NV];
    double Uc[NV];                                   // KU: conserved state of plane rz, own column
    bool sp_prev = false, sp_cur, sp_next;
    // fused CFL limit: split flags of plane rz-2 and the in-plane neighbours
    // of plane rz-1 decide whether the cell written next is a leaf that no
    // coarse-fine correction will change
    bool sp_prev2 = false, nxy_prev = false, nxy_cur = false;
    // fused CFL limit: cfl dx / max speed equals the minimum of cfl dx /
    // speed over the cells, bit for bit (both roundings are monotone), so
    // only the largest signal speed is kept
    double sp_max = 0.0;
    double nfs = 0.0;   // non-finite tracking of the folded limits
    double inv0 = 0.0;  // FP64: 1 / rho of the own column's plane rz (the predictor's)
    {
        double U[NV];
        bool sdummy;
        sp_cur = false;
        {
            load_u(a.uold, source_cell<GEN>(S, g, x, y, -2, sdummy), U);
            to_prim(U, a.gamma, Wm);
            load_u(a.uold, source_cell<GEN>(S, g, x, y, -1, sp_cur), U);
            inv0 = to_prim(U, a.gamma, W0);
            if constexpr (KU) copy5(Uc, U);
        }
        if (do_face) {
            load_u(a.uold, source_cell<GEN>(S, g, hx, hy, -1, sdummy), U);
            R Wh[NV];
            to_prim(U, a.gamma, Wh);
            lds_put(S.hw[2], lane, Wh);
        }
    }
    // FP64: ghost-ring cells are loaded one plane ahead of their use, so that
    // no wave waits for memory right before a barrier (the face-layer lanes
    // hold plane rz+1 for step 1 of iteration rz, the outer-ring and corner
    // lanes plane rz for step 2).  The mixed form keeps the registers this
    // costs: it runs more waves per SIMD instead.
    constexpr bool PF = sizeof(R) == 8;
    int rx = 0, ry = 0;
    const bool ring_role = do_outer || do_corner;
    if (do_corner) ring_pos(3, lane, rx, ry);
    else if (do_outer) ring_pos(2, lane, rx, ry);
    double Upf[NV];
    if constexpr (PF) {
        bool sdummy;
        if (do_face) load_u(a.uold, source_cell<GEN>(S, g, hx, hy, 0, sdummy), Upf);
        if (ring_role) load_u(a.uold, source_cell<GEN>(S, g, rx, ry, 0, sdummy), Upf);
    }
    // DB (NB = 2): planes alternate between two face buffers and split-flag
    // planes, so the fluxes of plane rz are read -- and plane rz is updated --
    // after the first barrier of the next iteration instead of after a third
    // barrier of their own; nothing written before a barrier of iteration
    // rz+1 is still being read from iteration rz-1 (the second barrier of
    // iteration rz separates them).  With one buffer the third barrier stays.
    constexpr bool DB = NB == 2;
    double Ucp[NV];   // DB with KU: conserved state of plane rz-1, own column
    // one buffer: partial update (uold + x and y flux differences) of plane
    // rz-1, in registers (FP64) or in the column's own LDS slot (mixed)
    constexpr bool ACC_LDS = sizeof(R) == 4;
    double acc_prev[NV], gz_prev[NV];
    R zp_prev[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        acc_prev[v] = 0.0;
        gz_prev[v] = 0.0;
        zp_prev[v] = R(0);
    }

    for (int rz = -1; rz <= ZC; ++rz) {
        const bool inner = rz >= 0 && rz < ZC;      // plane with x/y faces
        const int fb = DB ? (rz & 1) : 0;           // this plane's face buffer and split flags
        BrickFaces<R> &FB = S.u_[fb];
        uint8_t *spl = S.split[fb];
        double Un[NV];                               // conserved variables of plane rz+1, own column
        sp_next = false;
        load_u(a.uold, source_cell<GEN>(S, g, x, y, rz + 1, sp_next), Un);
        // 1. the reconstructed ghost ring: primitive variables of plane rz+1
        bool hsplit = false;
        if (do_face) {
            if (rz + 1 <= ZC) {
                R Wh[NV];
                bool sdummy;
                if constexpr (PF) {
                    to_prim(Upf, a.gamma, Wh);
                    if (rz + 2 <= ZC) load_u(a.uold, source_cell<GEN>(S, g, hx, hy, rz + 2, sdummy), Upf);
                } else {
                    double U[NV];
                    load_u(a.uold, source_cell<GEN>(S, g, hx, hy, rz + 1, sdummy), U);
                    to_prim(U, a.gamma, Wh);
                }
                lds_put(S.hw[(rz + 4) % 3], lane, Wh);
            }
            (void)source_cell<GEN>(S, g, hx, hy, rz, hsplit);
        }
        // 2. plane rz into LDS: W and split flags
        {
            lds_put(S.w, (x + 2) + PW * (y + 2), W0);
            if constexpr (GEN) spl[(x + 2) + PW * (y + 2)] = sp_cur;
        }
        if (do_face) {
            lds_put(S.w, (hx + 2) + PW * (hy + 2), ld5(S.hw[(rz + 3) % 3], lane).v);
            if constexpr (GEN) spl[(hx + 2) + PW * (hy + 2)] = hsplit;
        }
        if (ring_role && inner) {
            R Wr[NV];
            bool sdummy;
            if constexpr (PF) {
                to_prim(Upf, a.gamma, Wr);
                if (rz + 1 < ZC) load_u(a.uold, source_cell<GEN>(S, g, rx, ry, rz + 1, sdummy), Upf);
            } else {
                double U[NV];
                load_u(a.uold, source_cell<GEN>(S, g, rx, ry, rz, sdummy), U);
                to_prim(U, a.gamma, Wr);
            }
            lds_put(S.w, (rx + 2) + PW * (ry + 2), Wr);
        }
        __syncthreads();

        // 3. reconstruction of plane rz: the ghost ring first, then the own
        //    column, whose z face (rz-1 | rz) is evaluated at once
        if (do_face && inner) {
            R dW[3][NV], Wq[NV], st[NV];
            const int c = (hx + 2) + PW * (hy + 2);
            reconstruct<R>(ld5(S.hw[(rz + 3) % 3], lane).v, ld5(S.w, c - 1).v, ld5(S.w, c + 1).v, ld5(S.w, c - PW).v,
                           ld5(S.w, c + PW).v, ld5(S.hw[(rz + 2) % 3], lane).v, ld5(S.hw[(rz + 4) % 3], lane).v, h,
                           gam, dW, Wq);
            // x = -1 / y = -1 feed their high-side state to face (-1|0), x = 16
            // / y = 16 their low-side state to face (15|16)
            face_state<R>(Wq, hq < 2 ? dW[0] : dW[1], (hq & 1) == 0, st);
            ring_put(FB, hq, hk, st);
        }
        R sxm[NV], sym[NV];
        double gz[NV];
        double invp;
        {
            invp = to_prim(Un, a.gamma, Wp);
            R dW[3][NV], Wq[NV], st[NV], szm[NV];
            const int c = (x + 2) + PW * (y + 2);
            nxy_cur = GEN && (spl[c - 1] || spl[c + 1] || spl[c - PW] || spl[c + PW]);
            if constexpr (sizeof(R) == 8)
                reconstruct<R>(W0, ld5(S.w, c - 1).v, ld5(S.w, c + 1).v, ld5(S.w, c - PW).v, ld5(S.w, c + PW).v, Wm,
                               Wp, h, gam, R(inv0), dW, Wq);
            else
                reconstruct<R>(W0, ld5(S.w, c - 1).v, ld5(S.w, c + 1).v, ld5(S.w, c - PW).v, ld5(S.w, c + PW).v, Wm,
                               Wp, h, gam, dW, Wq);
            // written on every plane, also rz = -1 and 16 where nobody reads
            // them: the buffer of those planes is not in use then (plane
            // rz-2's update, the last reader of this buffer, ended before
            // the previous iteration's second barrier), and unconditional
            // code keeps the values out of branch merges
            face_state<R>(Wq, dW[0], true, st);
            lds_put(FB.fx, y * (BC + 1) + x + 1, st);
            face_state<R>(Wq, dW[1], true, st);
            lds_put(FB.fy, (y + 1) * BC + x, st);
            face_state<R>(Wq, dW[0], false, sxm);
            face_state<R>(Wq, dW[1], false, sym);
            face_state<R>(Wq, dW[2], false, szm);
            // at rz = -1 zp_prev is not a state (the result is discarded)
            face_G<GEN, R>(zp_prev, szm, gam, g1, r, sp_prev || sp_cur, gz);
            face_state<R>(Wq, dW[2], true, zp_prev);
        }
        // DB: plane rz-1 is complete: its x/y fluxes have been in the other
        // buffer since the barrier above, and its upper z face was just
        // evaluated.
        auto update_prev = [&]() {
            if constexpr (DB) {
                if (rz >= 1) {
                    const BrickFaces<R> &PB = S.u_[(rz - 1) & 1];
                    double Ucur[NV], out[NV];
                    if constexpr (KU) {
                        copy5(Ucur, Ucp);
                    } else {
                        bool sdummy;
                        load_u(a.uold, source_cell<GEN>(S, g, x, y, rz - 1, sdummy), Ucur);
                    }
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const double gxm = flux_G(PB.fx[v][y * (BC + 1) + x], r);
                        const double gxp = flux_G(PB.fx[v][y * (BC + 1) + x + 1], r);
                        const double gym = flux_G(PB.fy[v][y * BC + x], r);
                        const double gyp = flux_G(PB.fy[v][(y + 1) * BC + x], r);
                        const double acc = (Ucur[v] + (gxm - gxp)) + (gym - gyp);
                        out[v] = acc + (gz_prev[v] - gz[v]);
                    }
                    bool sdummy;
                    const int64_t cell = source_cell<GEN>(S, g, x, y, rz - 1, sdummy);
#pragma unroll
                    for (int v = 0; v < NV; ++v) a.unew[NV * cell + v] = out[v];
                    if (a.dt_next && !sp_prev && !(nxy_prev || sp_prev2 || sp_cur)) {
                        const double sp = signal_speed(out, a.gamma);
                        sp_max = sp > sp_max ? sp : sp_max;
                        track_finite(nfs, sp, out);
                    }
                }
            }
        };
        update_prev();
        __syncthreads();

        // 4. fluxes of the own low x and y faces, and of the x = 16 / y = 16
        //    faces on the extra lanes, each written over the face state it
        //    was computed from
        if (inner) {
            R F[NV];
            {
                face_F<GEN, R>(ld5(FB.fx, y * (BC + 1) + x).v, sxm, 0, gam, g1, GEN && (spl[(x + 1) + PW * (y + 2)] || sp_cur), F);
                store_flux(FB.fx, y * (BC + 1) + x, F, r);
                face_F<GEN, R>(ld5(FB.fy, y * BC + x).v, sym, 1, gam, g1, GEN && (spl[(x + 2) + PW * (y + 1)] || sp_cur), F);
                store_flux(FB.fy, y * BC + x, F, r);
            }
            if (extra_faces) {
                // ex = 0: face (15|16) of row hk, left state in fx, right in
                // sxm_hi; ex = 1: face (15|16) of column hk, fy and sym_hi;
                // flat indices into the buffer, so that both halves run as
                // one pass
                const int ex = lane >> 4;
                R *flat = &FB.fx[0][0];
                const int lb = ex ? NV * FXN + BC * BC + hk : hk * (BC + 1) + BC;
                const int ls = ex ? FYN : FXN;
                const int rb = NV * (FXN + FYN) + ex * NV * BC + hk;
                R Lf[NV], Rf[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Lf[v] = flat[lb + v * ls];
                    Rf[v] = flat[rb + v * BC];
                }
                const int s1 = ex ? (hk + 2) + PW * (BC + 1) : (BC + 1) + PW * (hk + 2);
                const int s2 = ex ? s1 + PW : s1 + 1;
                const bool z2 = GEN && (spl[s1] || spl[s2]);
                face_F<GEN, R>(Lf, Rf, ex, gam, g1, z2, F);
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    flat[lb + v * ls] = sizeof(R) == 8 ? static_cast<R>(static_cast<double>(F[v]) * r) : F[v];
            }
        }
        // DB: the fluxes are read after the next iteration's first barrier
        if constexpr (!DB) __syncthreads();

        // 5. update: plane rz-1 is complete; x/y part of plane rz
        if (!DB && rz >= 1) {
            double out[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                out[v] = (ACC_LDS ? S.acc[v][ACC_LDS ? tid : 0] : acc_prev[v]) + (gz_prev[v] - gz[v]);
            bool sdummy;
            const int64_t cell = source_cell<GEN>(S, g, x, y, rz - 1, sdummy);
#pragma unroll
            for (int v = 0; v < NV; ++v) a.unew[NV * cell + v] = out[v];
            if (a.dt_next && !sp_prev && !(nxy_prev || sp_prev2 || sp_cur)) {
                const double sp = signal_speed(out, a.gamma);
                sp_max = sp > sp_max ? sp : sp_max;
                track_finite(nfs, sp, out);
            }
        }
        if (!DB && inner) {
            double Ucur[NV];
            if constexpr (KU) {
                copy5(Ucur, Uc);
            } else {
                bool sdummy;
                load_u(a.uold, source_cell<GEN>(S, g, x, y, rz, sdummy), Ucur);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double gxm = flux_G(FB.fx[v][y * (BC + 1) + x], r);
                const double gxp = flux_G(FB.fx[v][y * (BC + 1) + x + 1], r);
                const double gym = flux_G(FB.fy[v][y * BC + x], r);
                const double gyp = flux_G(FB.fy[v][(y + 1) * BC + x], r);
                const double acc = (Ucur[v] + (gxm - gxp)) + (gym - gyp);
                if constexpr (ACC_LDS)
                    S.acc[v][tid] = acc;
                else
                    acc_prev[v] = acc;
            }
        }
        // shift the plane window
        {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                gz_prev[v] = rz >= 0 ? gz[v] : 0.0;
                Wm[v] = W0[v];
                W0[v] = Wp[v];
            }
            inv0 = invp;
            if constexpr (KU) {
                if constexpr (DB) copy5(Ucp, Uc);
                copy5(Uc, Un);
            }
        }
        sp_prev2 = sp_prev;
        sp_prev = sp_cur;
        sp_cur = sp_next;
        nxy_prev = nxy_cur;
    }
    if (a.dt_next) {
        double dt_min = nonfinite_limit(a.cfl * (a.dx / sp_max), nfs);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double o = __shfl_xor(dt_min, off, 64);
            dt_min = o < dt_min ? o : dt_min;
        }
        if (lane == 0) S.red[wave] = dt_min;
        __syncthreads();
        if (tid == 0) {
            double m = S.red[0];
            for (int k = 1; k < BT / 64; ++k) m = S.red[k] < m ? S.red[k] : m;
            fold_min(a.dt_next, m, a.hdr);
        }
    }
}

}  // namespace
}  // namespace rg

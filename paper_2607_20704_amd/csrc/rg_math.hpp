// rg_math.hpp -- per-cell and per-face arithmetic of the hydro update,
// shared by every kernel variant so that all of them produce the same bits.
//
// Paper Sec. 3: MUSCL-Hancock predictor-corrector with an HLLC Riemann
// solver.  The FP64 instances follow the CPU reference's expression order
// exactly (the library is built without FMA contraction); the float
// instances serve the mixed form.
#pragma once

#include "rg_internal.hpp"

namespace rg {

constexpr int NV = 5;

template <typename R> struct Math;

// Quotient and square root of positive normal doubles, correctly rounded.
// The general IEEE sequences first rescale operands whose exponents are
// extreme (near overflow, underflow or denormals) and afterwards patch the
// special values (zero, infinity, NaN); the operands of this update (density
// >= 1e-10, pressure >= 1e-20, signal speeds and mass fluxes of physical
// states) never need either, so only the arithmetic core is kept:
//   a / b: reciprocal estimate refined by two Newton-Raphson steps
//          y <- y + y (1 - b y), then q = a y and Markstein's correction
//          q <- q + y (a - b q) (P. Markstein, IBM J. Res. Dev. 34, 1990),
//          which with fused multiply-adds gives the correctly rounded
//          quotient;
//   sqrt:  reciprocal square root estimate y, then the coupled iteration of
//          g ~ sqrt(x) and h ~ 1/(2 sqrt(x)) (Goldschmidt): r = 1/2 - h g,
//          g <- g + g r, h <- h + h r, followed by two corrections
//          g <- g + h (x - g g).
// For such operands both give the same bits as a / b and sqrt(x); outside
// that range they stay within a few units in the last place (never used
// there).
__device__ __forceinline__ double div_pos(double a, double b)
{
    double y = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = a * y;
    const double rem = __builtin_fma(-b, q, a);
    return __builtin_fma(rem, y, q);
}

__device__ __forceinline__ double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
}

// madd(a, b, c) = a b + c: in double the product and the sum are rounded
// separately, exactly as the expression a * b + c (the library is built
// without contraction), so every double expression written with it keeps
// its bits; in float (the mixed form's reconstruction and Riemann solver) it
// is one fused multiply-add, one rounding and one instruction.
template <> struct Math<double> {
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt_pos(x); }
    static __device__ __forceinline__ double div(double a, double b) { return div_pos(a, b); }
    static __device__ __forceinline__ double madd(double a, double b, double c) { return a * b + c; }
};

template <> struct Math<float> {
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

// conservative -> primitive in double, floors applied; returns 1 / rho
// (of the floored density), which the predictor needs again
__device__ __forceinline__ double prim64(const double *U, double gamma, double *W)
{
    double rho = fmax(U[0], RG_RHO_MIN);
    double inv = div_pos(1.0, rho);
    double u = U[1] * inv;
    double v = U[2] * inv;
    double w = U[3] * inv;
    double q = (u * u + v * v) + w * w;
    double ek = 0.5 * rho * q;
    double p = fmax((gamma - 1.0) * (U[4] - ek), RG_P_MIN);
    W[0] = rho;
    W[1] = u;
    W[2] = v;
    W[3] = w;
    W[4] = p;
    return inv;
}

// Minmod of two undivided differences: zero unless a and b have the same
// strict sign, else the one of smaller magnitude.  Written as the median of
// (a, b, 0), which is exactly that value for every finite pair (only the
// sign of a zero result can differ): one v_med3 in float, four min/max in
// double, and no branches or lane-mask logic.
template <typename R> __device__ __forceinline__ R minmod(R a, R b);

template <> __device__ __forceinline__ float minmod<float>(float a, float b)
{
    return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}

template <> __device__ __forceinline__ double minmod<double>(double a, double b)
{
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Hancock half step W' = W - h sum_d A_d(W) dW_d (primitive Euler equations),
// inv = 1 / rho
template <typename R>
__device__ __forceinline__ void predict(const R *W, const R (*dW)[NV], R h, R gamma, R inv, R *Wp)
{
    const R rho = W[0], u = W[1], v = W[2], w = W[3], p = W[4];
    const R div = (dW[0][1] + dW[1][2]) + dW[2][3];
    // W'_k = W_k - h ((((u dW_x + v dW_y) + w dW_z) + s_k), the products and
    // sums in that order (each madd adds its product to the running sum)
    auto step = [&](int k, R base, R s) {
        const R t = Math<R>::madd(w, dW[2][k], Math<R>::madd(u, dW[0][k], v * dW[1][k]));
        return Math<R>::madd(-h, t + s, base);
    };
    Wp[0] = step(0, rho, rho * div);
    Wp[1] = step(1, u, dW[0][4] * inv);
    Wp[2] = step(2, v, dW[1][4] * inv);
    Wp[3] = step(3, w, dW[2][4] * inv);
    Wp[4] = step(4, p, (gamma * p) * div);
}

template <typename R>
__device__ __forceinline__ void predict(const R *W, const R (*dW)[NV], R h, R gamma, R *Wp)
{
    predict<R>(W, dW, h, gamma, Math<R>::div(R(1), W[0]), Wp);
}

// HLLC across a face normal to axis `dir`: Davis wave speeds, contact speed
// and star pressure in the form symmetric in the two sides, region chosen
// by S_L > 0, S* > 0, S_R > 0 in that order.  Computed branch-free: both
// candidate states are formed and one is selected.
template <typename R>
__device__ __forceinline__ void hllc(const R *WL, const R *WR, int dir, R gamma, R g1, R *F)
{
    // Both states are read once into registers and every choice below is a
    // choice between values: selecting or branching on pointers to the two
    // states (one may be in LDS, one private) would force the private state
    // into scratch memory.
    const R l0 = WL[0], l1 = WL[1], l2 = WL[2], l3 = WL[3], l4 = WL[4];
    const R r0 = WR[0], r1 = WR[1], r2 = WR[2], r3 = WR[3], r4 = WR[4];
    const R ul = dir == 0 ? l1 : (dir == 1 ? l2 : l3);
    const R ur = dir == 0 ? r1 : (dir == 1 ? r2 : r3);
    const R cl = Math<R>::sqrt_(Math<R>::div(gamma * l4, l0));
    const R cr = Math<R>::sqrt_(Math<R>::div(gamma * r4, r0));
    const R sl = fmin(ul - cl, ur - cr);
    const R sr = fmax(ul + cl, ur + cr);
    // u_L - S_L and S_R - u_R.  In float they are formed without the
    // cancellation of ul - sl, which in a cold flow (c below |u| / 2^24, as
    // where the pressure floor acts) rounds both to zero and makes the
    // division below infinite; algebraically the same values.  The double
    // instance keeps the reference's expressions (bit-equal results).
    R wl, wr;
    if constexpr (sizeof(R) == 4) {
        wl = fmax(cl, (ul - ur) + cr);
        wr = fmax((ul - ur) + cl, cr);
    } else {
        wl = ul - sl;
        wr = sr - ur;
    }
    const R ml = l0 * wl;
    const R mr = r0 * wr;
    const R inv = Math<R>::div(R(1), ml + mr);
    // ((mr ur + ml ul) + (pL - pR)) / (ml + mr) and
    // ((mr pL + ml pR) + ml mr (uL - uR)) / (ml + mr)
    const R sstar = (Math<R>::madd(mr, ur, ml * ul) + (l4 - r4)) * inv;
    const R pstar = Math<R>::madd(ml * mr, ul - ur, Math<R>::madd(mr, l4, ml * r4)) * inv;

    const bool useL = (sl > R(0)) || (sstar > R(0));
    const bool outer = useL ? (sl > R(0)) : !(sr > R(0));
    const R rho = useL ? l0 : r0, p = useL ? l4 : r4, un = useL ? ul : ur;
    const R w1 = useL ? l1 : r1, w2 = useL ? l2 : r2, w3 = useL ? l3 : r3;
    // the kinetic term of the chosen side only, from its selected velocities
    // (the same expression as per side, so the same value); forming one per
    // side let the compiler branch on the side to skip the other
    const R q = Math<R>::madd(w3, w3, Math<R>::madd(w1, w1, w2 * w2));
    const R s = useL ? sl : sr;
    const R E = Math<R>::madd(p, g1, (R(0.5) * rho) * q);
    const R d = Math<R>::div(R(1), s - sstar);
    // s - un = -(u_L - S_L) on the left, S_R - u_R on the right
    const R su = sizeof(R) == 4 ? (useL ? -wl : wr) : s - un;
    const R rs = outer ? rho : rho * su * d;
    const R es = outer ? E : Math<R>::madd(pstar, sstar, Math<R>::madd(su, E, -(p * un))) * d;
    const R ss = outer ? un : sstar;
    const R ps = outer ? p : pstar;
    const R m = rs * ss;
    F[0] = m;
    const R mp = Math<R>::madd(m, ss, ps);
    F[1] = dir == 0 ? mp : (m * w1);
    F[2] = dir == 1 ? mp : (m * w2);
    F[3] = dir == 2 ? mp : (m * w3);
    F[4] = (es + ps) * ss;
}


}  // namespace rg

namespace rg {

// minmod slopes along x, y, z of primitive cell W0 from its six neighbours
template <typename R>
__device__ __forceinline__ void slopes(const R *w0, const R *wxm, const R *wxp, const R *wym, const R *wyp,
                                       const R *wzm, const R *wzp, R (*dW)[NV])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        dW[0][v] = minmod<R>(w0[v] - wxm[v], wxp[v] - w0[v]);
        dW[1][v] = minmod<R>(w0[v] - wym[v], wyp[v] - w0[v]);
        dW[2][v] = minmod<R>(w0[v] - wzm[v], wzp[v] - w0[v]);
    }
}

// slopes, then the Hancock half step W'
template <typename R>
__device__ __forceinline__ void reconstruct(const R *w0, const R *wxm, const R *wxp, const R *wym, const R *wyp,
                                            const R *wzm, const R *wzp, R h, R gamma, R (*dW)[NV], R *Wp)
{
    slopes<R>(w0, wxm, wxp, wym, wyp, wzm, wzp, dW);
    predict<R>(w0, dW, h, gamma, Wp);
}

// the same with 1 / rho of W0 given (bit-identical: the same quotient)
template <typename R>
__device__ __forceinline__ void reconstruct(const R *w0, const R *wxm, const R *wxp, const R *wym, const R *wyp,
                                            const R *wzm, const R *wzp, R h, R gamma, R inv, R (*dW)[NV], R *Wp)
{
    slopes<R>(w0, wxm, wxp, wym, wyp, wzm, wzp, dW);
    predict<R>(w0, dW, h, gamma, inv, Wp);
}

// face state on the high (W' + dW/2) or low (W' - dW/2) side of a cell along
// one axis, density and pressure floored
template <typename R> __device__ __forceinline__ void face_state(const R *Wp, const R *dWa, bool high, R *st)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) st[v] = Math<R>::madd(high ? R(0.5) : R(-0.5), dWa[v], Wp[v]);
    st[0] = fmax(st[0], R(RG_RHO_MIN));
    st[4] = fmax(st[4], R(RG_P_MIN));
}

// LDS planes: a 5-variable quantity of many cells or faces stored as five
// planes a[v][i] (one per variable), so that the lanes of a wave, which
// handle consecutive i, touch consecutive words (40-byte records would put
// the words of neighbouring lanes 10 dwords apart and collide in the banks).
template <typename R, int N> __device__ __forceinline__ void lds_get(R *d, const R (&a)[NV][N], int i)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = a[v][i];
}

template <typename R, int N> __device__ __forceinline__ void lds_put(R (&a)[NV][N], int i, const R *src)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v][i] = src[v];
}

// the 5-variable value at index i of a plane set, in registers
template <typename R, int N> struct Ld5 {
    R v[NV];
    __device__ __forceinline__ Ld5(const R (&a)[NV][N], int i) { lds_get(v, a, i); }
};

template <typename R, int N> __device__ __forceinline__ Ld5<R, N> ld5(const R (&a)[NV][N], int i)
{
    return Ld5<R, N>(a, i);
}

// G = F dt/dx in double, or zero on a face touching a split cell
template <typename R> __device__ __forceinline__ void face_flux(const R *L, const R *Rt, int dir, R gamma, R g1,
                                                                double r, bool zero, double *G)
{
    R F[NV];
    hllc<R>(L, Rt, dir, gamma, g1, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) G[v] = zero ? 0.0 : static_cast<double>(F[v]) * r;
}

}  // namespace rg

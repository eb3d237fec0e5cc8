"""Reference solutions used to pin the oracle: nothing here calls the oracle or
the HIP library.

exact_riemann: the exact solution of the 1-D Riemann problem for an ideal gas
  (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4:
  Newton iteration on the pressure function, then sampling of the wave fan).
sedov_xi0: the dimensionless constant of the Sedov-Taylor point blast,
  R(t) = xi0 (E t^2 / rho0)^(1/5), from the similarity ODEs and the energy
  integral (as in Kamm & Timmes 2007, integrated numerically here).
"""
import math

import numpy as np
from scipy.integrate import solve_ivp


# ---------------------------------------------------------------------------
# exact Riemann solver
# ---------------------------------------------------------------------------

def _fk(p, rk, pk, ck, g):
    """Pressure function f_K(p) and its derivative (Toro eq. 4.6-4.7)."""
    if p > pk:                                   # shock
        A = 2.0 / ((g + 1.0) * rk)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    r = p / pk                                   # rarefaction
    f = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rk * ck) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


class ExactRiemann:
    def __init__(self, rl, ul, pl, rr, ur, pr, gamma):
        g = gamma
        self.g = g
        self.L = (rl, ul, pl, math.sqrt(g * pl / rl))
        self.R = (rr, ur, pr, math.sqrt(g * pr / rr))
        cl, cr = self.L[3], self.R[3]
        du = ur - ul
        p = max(1e-12, 0.5 * (pl + pr) - 0.125 * du * (rl + rr) * (cl + cr))   # PVRS guess
        for _ in range(100):
            fl, dfl = _fk(p, rl, pl, cl, g)
            fr, dfr = _fk(p, rr, pr, cr, g)
            pn = p - (fl + fr + du) / (dfl + dfr)
            pn = max(pn, 1e-14)
            if abs(pn - p) < 1e-15 * (pn + p):
                p = pn
                break
            p = pn
        fl, _ = _fk(p, rl, pl, cl, g)
        fr, _ = _fk(p, rr, pr, cr, g)
        self.pstar = p
        self.ustar = 0.5 * (ul + ur) + 0.5 * (fr - fl)
        self.rstar_l = self._rstar(self.L, p)
        self.rstar_r = self._rstar(self.R, p)

    def _rstar(self, K, p):
        rk, _, pk, _ = K
        g = self.g
        if p > pk:
            q = p / pk
            gm = (g - 1.0) / (g + 1.0)
            return rk * (q + gm) / (gm * q + 1.0)
        return rk * (p / pk) ** (1.0 / g)

    def shock_speed_right(self):
        rr, ur, pr, cr = self.R
        g = self.g
        return ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * self.pstar / pr + (g - 1.0) / (2.0 * g))

    def sample(self, s):
        """(rho, u, p) at x/t = s (array)."""
        s = np.asarray(s, np.float64)
        g = self.g
        out = np.empty((3,) + s.shape)
        for idx, x in np.ndenumerate(s):
            out[(slice(None),) + idx] = self._sample1(x, g)
        return out

    def _sample1(self, s, g):
        ps, us = self.pstar, self.ustar
        if s <= us:
            rk, uk, pk, ck = self.L
            if ps > pk:
                sh = uk - ck * math.sqrt((g + 1) / (2 * g) * ps / pk + (g - 1) / (2 * g))
                return (rk, uk, pk) if s <= sh else (self.rstar_l, us, ps)
            shl = uk - ck
            cs = ck * (ps / pk) ** ((g - 1) / (2 * g))
            stl = us - cs
            if s <= shl:
                return (rk, uk, pk)
            if s > stl:
                return (self.rstar_l, us, ps)
            c = 2.0 / (g + 1) * (ck + 0.5 * (g - 1) * (uk - s))
            r = rk * (c / ck) ** (2.0 / (g - 1))
            u = 2.0 / (g + 1) * (ck + 0.5 * (g - 1) * uk + s)
            return (r, u, pk * (c / ck) ** (2 * g / (g - 1)))
        rk, uk, pk, ck = self.R
        if ps > pk:
            sh = uk + ck * math.sqrt((g + 1) / (2 * g) * ps / pk + (g - 1) / (2 * g))
            return (rk, uk, pk) if s >= sh else (self.rstar_r, us, ps)
        shr = uk + ck
        cs = ck * (ps / pk) ** ((g - 1) / (2 * g))
        str_ = us + cs
        if s >= shr:
            return (rk, uk, pk)
        if s < str_:
            return (self.rstar_r, us, ps)
        c = 2.0 / (g + 1) * (ck - 0.5 * (g - 1) * (uk - s))
        r = rk * (c / ck) ** (2.0 / (g - 1))
        u = 2.0 / (g + 1) * (-ck + 0.5 * (g - 1) * uk + s)
        return (r, u, pk * (c / ck) ** (2 * g / (g - 1)))


# ---------------------------------------------------------------------------
# Sedov-Taylor constant
# ---------------------------------------------------------------------------

def sedov_xi0(gamma, alpha=0.4):
    """xi0 for a spherical blast in uniform gas.

    With v = (r/t) U(xi), rho = rho0 G(xi), c^2 = (r/t)^2 Z(xi), xi = r/R(t),
    R ~ t^alpha (alpha = 2/5), the Euler equations (mass, momentum, entropy)
    become three linear equations for G', U', Z' (derivatives in ln xi):
        (U-a) G' + G U'                 = -3 G U
        Z/(g G) G' + (U-a) U' + Z'/g    = U - U^2 - 2 Z/g
        (1-g)(U-a)/G G' + (U-a)/Z Z'    = -2 (U - 1)
    started from the strong-shock values at xi = 1 and integrated inward.
    The energy E = 4 pi rho0 R^5 / t^2 * I with
        I = int_0^1 xi^4 G (U^2/2 + Z/(g(g-1))) dxi
    gives xi0 = (4 pi I)^(-1/5)."""
    g, a = gamma, alpha

    def rhs(s, y):
        G, U, Z = y
        M = np.array([[U - a, G, 0.0],
                      [Z / (g * G), U - a, 1.0 / g],
                      [(1.0 - g) * (U - a) / G, 0.0, (U - a) / Z]])
        b = np.array([-3.0 * G * U, U - U * U - 2.0 * Z / g, -2.0 * (U - 1.0)])
        return np.linalg.solve(M, b)

    y0 = [(g + 1.0) / (g - 1.0), 2.0 * a / (g + 1.0), 2.0 * g * (g - 1.0) * a * a / (g + 1.0) ** 2]
    # pressure tends to a constant at the centre, so the integrand falls at
    # least like xi^2 there; stopping at xi = e^-6 changes I by < 1e-6 relative
    s_end = -6.0
    sol = solve_ivp(rhs, (0.0, s_end), y0, rtol=1e-10, atol=1e-13, dense_output=True, method="DOP853")
    if not sol.success:
        raise RuntimeError(sol.message)
    s = np.linspace(0.0, s_end, 20001)
    G, U, Z = sol.sol(s)
    xi = np.exp(s)
    integrand = xi ** 4 * G * (0.5 * U * U + Z / (g * (g - 1.0)))
    I = -np.trapezoid(integrand, xi)
    return (4.0 * math.pi * I) ** (-0.2)

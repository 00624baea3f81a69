"""Exact solution of the 1D special-relativistic hydrodynamic Riemann problem
(zero tangential velocity, ideal gas), after Marti & Mueller, J. Fluid Mech.
258, 317 (1994) and Living Rev. Relativ. 6, 7 (2003).

Independent of the oracle: used only to pin the oracle's full scheme on the
relativistic shock tube of section 3.1.2 of the Gmunu paper.

States are (rho, p, v).  The star pressure is the root of
v_L*(p) - v_R*(p), where each side is joined to the star region by a shock
(Taub adiabat + Rankine-Hugoniot jump) or a rarefaction (constant Riemann
invariant along an isentrope).
"""
from __future__ import annotations

import math

from scipy.optimize import brentq


def _h(rho, p, g):
    return 1.0 + g / (g - 1.0) * p / rho


def _cs(rho, p, g):
    return math.sqrt(g * p / (rho * _h(rho, p, g))) if p > 0 else 0.0


def _A(c, g):
    s = math.sqrt(g - 1.0)
    return (s + c) / (s - c)


def _raref_v(state, pb, g, sign):
    """Velocity behind a rarefaction reached from `state` at pressure pb.
    sign = -1 for a left-moving wave (J+ constant), +1 for a right-moving one."""
    rho, p, v = state
    rhob = rho * (pb / p) ** (1.0 / g)
    ca, cb = _cs(rho, p, g), _cs(rhob, pb, g)
    s = math.sqrt(g - 1.0)
    # ln((1+v)/(1-v)) changes by -sign * (2/s) [ln A(c_a) - ln A(c_b)]
    lnz = math.log((1.0 + v) / (1.0 - v)) - sign * (2.0 / s) * (math.log(_A(ca, g)) - math.log(_A(cb, g)))
    z = math.exp(lnz)
    return (z - 1.0) / (z + 1.0)


def _taub_h(state, pb, g):
    """Post-shock specific enthalpy on the Taub adiabat for an ideal gas."""
    rho, p, v = state
    ha = _h(rho, p, g)
    k = (g - 1.0) * (p - pb) / (g * pb)
    a = 1.0 + k
    b = -k
    c = ha * (p - pb) / rho - ha * ha
    return (-b + math.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)


def _shock(state, pb, g, sign):
    """(v_b, rho_b, V_shock) behind a shock of pressure pb into `state`.
    sign = -1: shock moving left (left state), +1: moving right."""
    rho, p, v = state
    ha = _h(rho, p, g)
    hb = _taub_h(state, pb, g)
    rhob = g * pb / ((g - 1.0) * (hb - 1.0))
    j2 = (pb - p) / (ha / rho - hb / rhob)
    j = sign * math.sqrt(j2)
    Wa = 1.0 / math.sqrt(1.0 - v * v)
    r2w2 = rho * rho * Wa * Wa
    Vs = (r2w2 * v + j * math.sqrt(j2 + r2w2 * (1.0 - v * v))) / (r2w2 + j2)
    Ws = 1.0 / math.sqrt(1.0 - Vs * Vs)
    vb = (ha * Wa * v + Ws * (pb - p) / j) / (ha * Wa + (pb - p) * (Ws * v / j + 1.0 / (rho * Wa)))
    return vb, rhob, Vs


def _vstar(state, pb, g, sign):
    if pb > state[1]:
        return _shock(state, pb, g, sign)[0]
    if pb == state[1]:
        return state[2]
    return _raref_v(state, pb, g, sign)


class RiemannSRHD:
    def __init__(self, left, right, gamma):
        self.L, self.R, self.g = tuple(left), tuple(right), gamma
        g = gamma
        f = lambda pp: _vstar(self.L, pp, g, -1) - _vstar(self.R, pp, g, +1)
        lo = 1e-14 * max(self.L[1], self.R[1])
        hi = 10.0 * max(self.L[1], self.R[1]) + 1.0
        self.ps = brentq(f, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        self.vs = _vstar(self.L, self.ps, g, -1)
        # left wave
        if self.ps > self.L[1]:
            _, self.rhoL, self.VL = _shock(self.L, self.ps, g, -1)
            self.left_shock = True
        else:
            self.rhoL = self.L[0] * (self.ps / self.L[1]) ** (1.0 / g)
            self.left_shock = False
        if self.ps > self.R[1]:
            _, self.rhoR, self.VR = _shock(self.R, self.ps, g, +1)
            self.right_shock = True
        else:
            self.rhoR = self.R[0] * (self.ps / self.R[1]) ** (1.0 / g) if self.R[1] > 0 else 0.0
            self.right_shock = False

    def _fan(self, state, xi, sign):
        """State inside a rarefaction fan at similarity coordinate xi."""
        g = self.g
        rho, p, v = state

        def speed(pp):
            vb = _raref_v(state, pp, g, sign)
            rb = rho * (pp / p) ** (1.0 / g)
            c = _cs(rb, pp, g)
            return (vb + sign * c) / (1.0 + sign * vb * c)

        pp = brentq(lambda x: speed(x) - xi, self.ps, p, xtol=1e-15, rtol=1e-15, maxiter=500)
        return rho * (pp / p) ** (1.0 / g), pp, _raref_v(state, pp, g, sign)

    def sample(self, xi):
        """(rho, p, v) at x/t = xi."""
        g = self.g
        L, R = self.L, self.R
        if xi < self.vs:
            if self.left_shock:
                return L if xi < self.VL else (self.rhoL, self.ps, self.vs)
            cL = _cs(L[0], L[1], g)
            head = (L[2] - cL) / (1.0 - L[2] * cL)
            cs = _cs(self.rhoL, self.ps, g)
            tail = (self.vs - cs) / (1.0 - self.vs * cs)
            if xi < head:
                return L
            if xi > tail:
                return (self.rhoL, self.ps, self.vs)
            return self._fan(L, xi, -1)
        if self.right_shock:
            return R if xi > self.VR else (self.rhoR, self.ps, self.vs)
        cR = _cs(R[0], R[1], g)
        head = (R[2] + cR) / (1.0 + R[2] * cR)
        cs = _cs(self.rhoR, self.ps, g)
        tail = (self.vs + cs) / (1.0 + self.vs * cs)
        if xi > head:
            return R
        if xi < tail:
            return (self.rhoR, self.ps, self.vs)
        return self._fan(R, xi, +1)

    def cell_average(self, x0, x1, t, x_jump, nsub=64):
        """Density, pressure, velocity averaged over [x0, x1] at time t."""
        acc = [0.0, 0.0, 0.0]
        for s in range(nsub):
            x = x0 + (s + 0.5) * (x1 - x0) / nsub
            st = self.sample((x - x_jump) / t)
            for k in range(3):
                acc[k] += st[k] / nsub
        return tuple(acc)


def jump_residuals(state_a, pb, gamma, sign):
    """Rankine-Hugoniot residuals [U (v - V) + F-part] across the shock of
    pressure pb into state_a: mass, momentum and energy, each relative."""
    va_b, rhob, Vs = _shock(state_a, pb, gamma, sign)
    res = []
    for (rho, p, v) in (state_a, (rhob, pb, va_b)):
        W = 1.0 / math.sqrt(1.0 - v * v)
        h = _h(rho, p, gamma)
        D = rho * W
        S = rho * h * W * W * v
        E = rho * h * W * W - p
        res.append(((D * (v - Vs),), (S * (v - Vs), p), (E * (v - Vs), p * v)))
    a, b = res
    out = []
    for k in range(3):
        scale = max(abs(x) for x in a[k] + b[k])
        out.append(abs(sum(a[k]) - sum(b[k])) / max(scale, 1e-300))
    return out

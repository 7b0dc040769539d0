"""Exact solution of the Riemann problem for the 1-D Euler equations.

TEST INFRASTRUCTURE ONLY (the analytical solution the paper compares its
shock-tube results with, Sec. V.C-D).  Derived from the Euler equations for
an ideal gas p = (gamma - 1) rho e:

* across a shock the Rankine-Hugoniot conditions give the velocity jump
  f_K(p) = (p - p_K) sqrt(A_K / (p + B_K)), A_K = 2 / ((gamma+1) rho_K),
  B_K = p_K (gamma-1)/(gamma+1);
* across a rarefaction the Riemann invariant u +- 2c/(gamma-1) and the
  isentrope p / rho^gamma are constant, so
  f_K(p) = 2 c_K/(gamma-1) [(p/p_K)^((gamma-1)/(2 gamma)) - 1];
* the star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 (monotone in p,
  found by bisection refined with Newton steps), u* = (u_L + u_R + f_R - f_L)/2.

Each side may hold its own gas (gamma_L, gamma_R): every wave lies inside
one gas and the contact separates them, so f_K uses the gamma of side K.

The solution is self-similar in s = (x - x_d) / t.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho_k, p_k, c_k, g):
    if p > p_k:
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        return (p - p_k) * s, s * (1.0 - 0.5 * (p - p_k) / (p + B))
    r = p / p_k
    ex = (g - 1.0) / (2.0 * g)
    return 2.0 * c_k / (g - 1.0) * (r ** ex - 1.0), (1.0 / (rho_k * c_k)) * r ** (-(g + 1.0) / (2.0 * g))


class RiemannSolution:
    """Exact solution for left/right states (rho, u, p) and gamma, or a pair
    (gamma_L, gamma_R) for two gases."""

    def __init__(self, left, right, gamma=1.4):
        gl, gr = (float(gamma[0]), float(gamma[1])) if isinstance(gamma, (tuple, list)) else (float(gamma),) * 2
        self.gl, self.gr = gl, gr
        self.rl, self.ul, self.pl = map(float, left)
        self.rr, self.ur, self.pr = map(float, right)
        self.cl = math.sqrt(gl * self.pl / self.rl)
        self.cr = math.sqrt(gr * self.pr / self.rr)
        du = self.ur - self.ul
        if 2.0 * self.cl / (gl - 1.0) + 2.0 * self.cr / (gr - 1.0) <= du:
            raise ValueError("vacuum is generated; not handled")

        def F(p):
            fl, dfl = _f_and_df(p, self.rl, self.pl, self.cl, gl)
            fr, dfr = _f_and_df(p, self.rr, self.pr, self.cr, gr)
            return fl + fr + du, dfl + dfr

        lo, hi = 1e-14, max(self.pl, self.pr)
        while F(hi)[0] < 0.0:
            hi *= 2.0
        for _ in range(200):  # bisection to a bracket, then Newton
            mid = 0.5 * (lo + hi)
            if F(mid)[0] < 0.0:
                lo = mid
            else:
                hi = mid
            if hi - lo < 1e-6 * hi:
                break
        p = 0.5 * (lo + hi)
        for _ in range(50):
            val, der = F(p)
            pn = p - val / der
            if not (lo <= pn <= hi):
                pn = 0.5 * (lo + hi)
            if F(pn)[0] < 0.0:
                lo = pn
            else:
                hi = pn
            if abs(pn - p) <= 1e-15 * p:
                p = pn
                break
            p = pn
        self.p_star = p
        fl, _ = _f_and_df(p, self.rl, self.pl, self.cl, gl)
        fr, _ = _f_and_df(p, self.rr, self.pr, self.cr, gr)
        self.u_star = 0.5 * (self.ul + self.ur) + 0.5 * (fr - fl)
        # left wave (gas of the left side)
        g = gl
        gm = (g - 1.0) / (g + 1.0)
        if p > self.pl:
            self.rho_star_l = self.rl * (p / self.pl + gm) / (gm * p / self.pl + 1.0)
            self.s_l = self.ul - self.cl * math.sqrt((g + 1.0) / (2.0 * g) * p / self.pl + (g - 1.0) / (2.0 * g))
            self.left_shock = True
        else:
            self.rho_star_l = self.rl * (p / self.pl) ** (1.0 / g)
            self.c_star_l = self.cl * (p / self.pl) ** ((g - 1.0) / (2.0 * g))
            self.head_l = self.ul - self.cl
            self.tail_l = self.u_star - self.c_star_l
            self.left_shock = False
        # right wave (gas of the right side)
        g = gr
        gm = (g - 1.0) / (g + 1.0)
        if p > self.pr:
            self.rho_star_r = self.rr * (p / self.pr + gm) / (gm * p / self.pr + 1.0)
            self.s_r = self.ur + self.cr * math.sqrt((g + 1.0) / (2.0 * g) * p / self.pr + (g - 1.0) / (2.0 * g))
            self.right_shock = True
        else:
            self.rho_star_r = self.rr * (p / self.pr) ** (1.0 / g)
            self.c_star_r = self.cr * (p / self.pr) ** ((g - 1.0) / (2.0 * g))
            self.head_r = self.ur + self.cr
            self.tail_r = self.u_star + self.c_star_r
            self.right_shock = False

    def sample(self, s):
        """(rho, u, p) at similarity coordinates s = (x - x_d) / t (array)."""
        g = self.gl
        s = np.asarray(s, dtype=np.float64)
        rho = np.empty_like(s)
        u = np.empty_like(s)
        p = np.empty_like(s)
        left = s <= self.u_star
        # left side of the contact
        if self.left_shock:
            a = left & (s < self.s_l)
            b = left & (s >= self.s_l)
            rho[a], u[a], p[a] = self.rl, self.ul, self.pl
            rho[b], u[b], p[b] = self.rho_star_l, self.u_star, self.p_star
        else:
            a = left & (s < self.head_l)
            b = left & (s >= self.tail_l)
            f = left & (s >= self.head_l) & (s < self.tail_l)
            rho[a], u[a], p[a] = self.rl, self.ul, self.pl
            rho[b], u[b], p[b] = self.rho_star_l, self.u_star, self.p_star
            uf = 2.0 / (g + 1.0) * (self.cl + (g - 1.0) / 2.0 * self.ul + s[f])
            cf = 2.0 / (g + 1.0) * (self.cl + (g - 1.0) / 2.0 * (self.ul - s[f]))
            rho[f] = self.rl * (cf / self.cl) ** (2.0 / (g - 1.0))
            u[f] = uf
            p[f] = self.pl * (cf / self.cl) ** (2.0 * g / (g - 1.0))
        right = ~left
        g = self.gr
        if self.right_shock:
            a = right & (s > self.s_r)
            b = right & (s <= self.s_r)
            rho[a], u[a], p[a] = self.rr, self.ur, self.pr
            rho[b], u[b], p[b] = self.rho_star_r, self.u_star, self.p_star
        else:
            a = right & (s > self.head_r)
            b = right & (s <= self.tail_r)
            f = right & (s > self.tail_r) & (s <= self.head_r)
            rho[a], u[a], p[a] = self.rr, self.ur, self.pr
            rho[b], u[b], p[b] = self.rho_star_r, self.u_star, self.p_star
            uf = 2.0 / (g + 1.0) * (-self.cr + (g - 1.0) / 2.0 * self.ur + s[f])
            cf = 2.0 / (g + 1.0) * (self.cr - (g - 1.0) / 2.0 * (self.ur - s[f]))
            rho[f] = self.rr * (cf / self.cr) ** (2.0 / (g - 1.0))
            u[f] = uf
            p[f] = self.pr * (cf / self.cr) ** (2.0 * g / (g - 1.0))
        return rho, u, p

    def profile(self, x, x_d: float, t: float):
        return self.sample((np.asarray(x, dtype=np.float64) - x_d) / t)


def l1_error(values, exact, dx: float) -> float:
    """Discrete L1 norm dx * sum |values - exact|."""
    return float(dx * np.sum(np.abs(np.asarray(values) - np.asarray(exact))))

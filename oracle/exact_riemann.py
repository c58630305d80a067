"""Exact solution of the 1D Riemann problem for an ideal gas.

TEST INFRASTRUCTURE ONLY (part of the oracle): used to score the
shock-tube run; nothing in the product path imports it.

The paper validates its solver on Sod's shock tube ("Tuning Experiments",
convergence-test initial conditions) and cites Toro's textbook for the
method.  This module follows the textbook construction: the star-region
pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where for side K

  rarefaction (p <= p_K): f_K = 2 c_K / (gamma-1) * ((p/p_K)^((gamma-1)/(2 gamma)) - 1)
  shock       (p >  p_K): f_K = (p - p_K) * sqrt(A_K / (p + B_K)),
                          A_K = 2 / ((gamma+1) rho_K), B_K = (gamma-1)/(gamma+1) p_K,

then u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2, and the self-similar
solution is sampled at x/t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class Side:
    rho: float
    u: float
    p: float


def _sound(gamma: float, s: Side) -> float:
    return math.sqrt(gamma * s.p / s.rho)


def _f_and_df(gamma: float, p: float, s: Side) -> tuple[float, float]:
    c = _sound(gamma, s)
    if p <= s.p:
        pr = p / s.p
        f = 2.0 * c / (gamma - 1.0) * (pr ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = (1.0 / (s.rho * c)) * pr ** (-(gamma + 1.0) / (2.0 * gamma))
    else:
        a = 2.0 / ((gamma + 1.0) * s.rho)
        b = (gamma - 1.0) / (gamma + 1.0) * s.p
        q = math.sqrt(a / (p + b))
        f = (p - s.p) * q
        df = q * (1.0 - 0.5 * (p - s.p) / (b + p))
    return f, df


def star_state(gamma: float, left: Side, right: Side, tol: float = 1e-14) -> tuple[float, float]:
    """Return (p*, u*) by Newton iteration on the pressure function."""
    cl, cr = _sound(gamma, left), _sound(gamma, right)
    du = right.u - left.u
    if 2.0 * (cl + cr) / (gamma - 1.0) <= du:
        raise ValueError("initial data generate vacuum")
    # two-rarefaction guess, clipped to be positive
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((cl + cr - 0.5 * (gamma - 1.0) * du) /
         (cl / left.p ** z + cr / right.p ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(200):
        fl, dfl = _f_and_df(gamma, p, left)
        fr, dfr = _f_and_df(gamma, p, right)
        g = fl + fr + du
        pn = p - g / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(gamma, p, left)
    fr, _ = _f_and_df(gamma, p, right)
    u = 0.5 * (left.u + right.u) + 0.5 * (fr - fl)
    return p, u


@dataclass(frozen=True)
class Waves:
    p_star: float
    u_star: float
    rho_star_l: float
    rho_star_r: float
    # characteristic speeds (the ones that exist for this configuration)
    left_head: float
    left_tail: float
    right_head: float
    right_tail: float
    left_is_shock: bool
    right_is_shock: bool


def waves(gamma: float, left: Side, right: Side) -> Waves:
    ps, us = star_state(gamma, left, right)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    cl, cr = _sound(gamma, left), _sound(gamma, right)
    if ps > left.p:  # left shock
        r = ps / left.p
        rsl = left.rho * (r + g1) / (g1 * r + 1.0)
        sl = left.u - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * r + (gamma - 1.0) / (2.0 * gamma))
        lh = lt = sl
        lshock = True
    else:
        rsl = left.rho * (ps / left.p) ** (1.0 / gamma)
        csl = cl * (ps / left.p) ** ((gamma - 1.0) / (2.0 * gamma))
        lh, lt = left.u - cl, us - csl
        lshock = False
    if ps > right.p:  # right shock
        r = ps / right.p
        rsr = right.rho * (r + g1) / (g1 * r + 1.0)
        sr = right.u + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * r + (gamma - 1.0) / (2.0 * gamma))
        rh = rt = sr
        rshock = True
    else:
        rsr = right.rho * (ps / right.p) ** (1.0 / gamma)
        csr = cr * (ps / right.p) ** ((gamma - 1.0) / (2.0 * gamma))
        rh, rt = right.u + cr, us + csr
        rshock = False
    return Waves(ps, us, rsl, rsr, lh, lt, rh, rt, lshock, rshock)


def sample(gamma: float, left: Side, right: Side, s: float) -> tuple[float, float, float]:
    """(rho, u, p) of the self-similar solution at s = (x - x0)/t."""
    w = waves(gamma, left, right)
    cl, cr = _sound(gamma, left), _sound(gamma, right)
    if s <= w.u_star:  # left of the contact
        if w.left_is_shock:
            if s <= w.left_head:
                return left.rho, left.u, left.p
            return w.rho_star_l, w.u_star, w.p_star
        if s <= w.left_head:
            return left.rho, left.u, left.p
        if s >= w.left_tail:
            return w.rho_star_l, w.u_star, w.p_star
        # inside the left rarefaction fan
        a = 2.0 / (gamma + 1.0)
        b = (gamma - 1.0) / ((gamma + 1.0) * cl)
        c = a + b * (left.u - s)
        rho = left.rho * c ** (2.0 / (gamma - 1.0))
        u = a * (cl + 0.5 * (gamma - 1.0) * left.u + s)
        p = left.p * c ** (2.0 * gamma / (gamma - 1.0))
        return rho, u, p
    if w.right_is_shock:
        if s >= w.right_head:
            return right.rho, right.u, right.p
        return w.rho_star_r, w.u_star, w.p_star
    if s >= w.right_head:
        return right.rho, right.u, right.p
    if s <= w.right_tail:
        return w.rho_star_r, w.u_star, w.p_star
    a = 2.0 / (gamma + 1.0)
    b = (gamma - 1.0) / ((gamma + 1.0) * cr)
    c = a - b * (right.u - s)
    rho = right.rho * c ** (2.0 / (gamma - 1.0))
    u = a * (-cr + 0.5 * (gamma - 1.0) * right.u + s)
    p = right.p * c ** (2.0 * gamma / (gamma - 1.0))
    return rho, u, p


def sample_cells(gamma: float, left: Side, right: Side, x0: float, t: float, xs) -> list[tuple[float, float, float]]:
    """Exact (rho, u, p) at the points xs at time t > 0."""
    return [sample(gamma, left, right, (x - x0) / t) for x in xs]

"""Floating-point operations of the method itself, per cell-update.

MEASUREMENT INFRASTRUCTURE, not a parity reference: it gives the work figure
behind the benchmark's ALU roofline.  Only tests and the benchmark's
bookkeeping read it; the product path never does.

The oracle's counting build (flopcount.cpp) counts the oracle's own code,
which is written for checking by eye and recomputes on purpose: every cell's
limited slope is formed twice per axis (once for each face it touches), the
conserved form of each face state is formed again inside the physical flux,
and both sides' fluxes are formed before the HLLC branch is chosen.  What the
scheme needs (paper, section "Tuning Experiments / The Target Program": the
state-vector equations, the Interpolate equation, the HLLC flux, AddFlux, the
two-stage time marching and the CFL time step) is less, and that is counted
here, by running one step of the scheme on a counting number type with every
quantity formed once:

  * V(U) once per cell and stage: 1/rho, v_a = m_a/rho, p = (gamma-1)(E - v.m/2);
  * one difference per face and primitive, one limited half-slope per cell,
    axis and primitive, and the two face values y -+ slope/2 of the cell;
  * per face one HLLC solve that picks its branch from the Davis speeds and
    the contact speed first and then forms the physical flux, the conserved
    face state and the star state of the one side it uses;
  * AddFlux: per field and axis one difference of face fluxes, one product
    with c dt/dr_a (a folded constant) and one sum;
  * the CFL term of the new state: V(U), c = sqrt(gamma p / rho) and
    sum_a (|v_a| + c)/dr_a with 1/dr_a folded.

Counted: additions, subtractions, multiplications, divisions and square
roots (one each; a fused multiply-add counts two).  Not counted: negation,
comparisons, minimum, maximum and absolute value (the limiter, the Davis
speeds and the HLLC branch are made of these).  Constants of a mesh
(gamma - 1, 1/(gamma - 1), gamma, c dt/dr_a, 1/dr_a, 1/2) are folded.
"""
from __future__ import annotations

import math

import numpy as np


class Counter:
    def __init__(self):
        self.add = self.mul = self.div = self.sqrt = 0

    @property
    def total(self) -> int:
        return self.add + self.mul + self.div + self.sqrt


_C = Counter()


class F:
    """A float whose arithmetic is counted in the module's counter."""
    __slots__ = ("v",)

    def __init__(self, v):
        self.v = float(v.v if isinstance(v, F) else v)

    def __add__(self, o):
        _C.add += 1
        return F(self.v + _val(o))

    __radd__ = __add__

    def __sub__(self, o):
        _C.add += 1
        return F(self.v - _val(o))

    def __rsub__(self, o):
        _C.add += 1
        return F(_val(o) - self.v)

    def __mul__(self, o):
        _C.mul += 1
        return F(self.v * _val(o))

    __rmul__ = __mul__

    def __truediv__(self, o):
        _C.div += 1
        return F(self.v / _val(o))

    def __rtruediv__(self, o):
        _C.div += 1
        return F(_val(o) / self.v)

    def __neg__(self):
        return F(-self.v)


def _val(x):
    return x.v if isinstance(x, F) else float(x)


def fsqrt(x: F) -> F:
    _C.sqrt += 1
    return F(math.sqrt(x.v))


def minmod(a: F, b: F) -> F:
    """The minbee limiter: 0 where the signs differ or one is 0, else the smaller magnitude."""
    if (a.v > 0.0 and b.v > 0.0) or (a.v < 0.0 and b.v < 0.0):
        return a if abs(a.v) < abs(b.v) else b
    return F(0.0)


class Gas:
    def __init__(self, gamma: float):
        self.gamma = gamma
        self.gm1 = gamma - 1.0
        self.inv_gm1 = 1.0 / (gamma - 1.0)


def prim_of_cons(d: int, g: Gas, u: list) -> list:
    """rho, v_a, p from rho, m_a, E: one division, then products."""
    inv = 1.0 / u[0]
    v = [u[1 + a] * inv for a in range(d)]
    vm = v[0] * u[1]
    for a in range(1, d):
        vm = vm + v[a] * u[1 + a]
    p = (u[d + 1] - 0.5 * vm) * g.gm1
    return [u[0]] + v + [p]


def hllc(d: int, g: Gas, ax: int, vl: list, vr: list) -> list:
    """HLLC flux with Davis speeds; the branch is chosen before any flux is formed and
    only the side it uses is evaluated."""
    rl, rr = vl[0], vr[0]
    ul, ur = vl[1 + ax], vr[1 + ax]
    pl, pr = vl[d + 1], vr[d + 1]
    cl = fsqrt(g.gamma * pl / rl)
    cr = fsqrt(g.gamma * pr / rr)
    a1, a2 = ul - cl, ur - cr
    sl = a1 if a1.v < a2.v else a2
    b1, b2 = ul + cl, ur + cr
    sr = b1 if b1.v > b2.v else b2

    def side(v, with_state):
        """Physical flux of one face state, and its conserved state if asked for."""
        r, un, p = v[0], v[1 + ax], v[d + 1]
        mn = r * un
        v2 = un * un
        for b in range(d):
            if b != ax:
                v2 = v2 + v[1 + b] * v[1 + b]
        E = p * g.inv_gm1 + (0.5 * r) * v2
        flux = [mn] + [mn * un + p if b == ax else mn * v[1 + b] for b in range(d)] + [(E + p) * un]
        if not with_state:
            return flux, None
        mom = [mn if b == ax else r * v[1 + b] for b in range(d)]
        return flux, [r] + mom + [E]

    if sl.v >= 0.0:
        return side(vl, False)[0]
    if sr.v <= 0.0:
        return side(vr, False)[0]
    al, ar = sl - ul, sr - ur
    ral, rar = rl * al, rr * ar
    sstar = (pr - pl + ral * ul - rar * ur) / (ral - rar)
    if sstar.v >= 0.0:
        v, sk, rak = vl, sl, ral
    else:
        v, sk, rak = vr, sr, rar
    fk, uk = side(v, True)
    r, un, p = v[0], v[1 + ax], v[d + 1]
    fac = rak / (sk - sstar)
    ust = [fac] + [fac * sstar if b == ax else fac * v[1 + b] for b in range(d)]
    ust.append(fac * (uk[d + 1] / r + (sstar - un) * (sstar + p / rak)))
    return [fk[q] + sk * (ust[q] - uk[q]) for q in range(d + 2)]


def _shift(i, n):
    return i % n


def stage(d: int, g: Gas, n: tuple, Uin: list, Ubase: list, coefs: list) -> list:
    """One stage on a periodic mesh; U[q] is a flat list of F over cells (x fastest)."""
    nf = d + 2
    ncell = n[0] * n[1] * n[2]
    V = [prim_of_cons(d, g, [Uin[q][c] for q in range(nf)]) for c in range(ncell)]
    strides = [1, n[0], n[0] * n[1]]

    def idx(c, ax, off):
        i = [c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]
        i[ax] = _shift(i[ax] + off, n[ax])
        return i[0] + n[0] * (i[1] + n[1] * i[2])

    acc = [[None] * ncell for _ in range(nf)]
    for ax in range(d):
        # one difference per face (the face below each cell) and primitive
        diff = [[V[c][q] - V[idx(c, ax, -1)][q] for c in range(ncell)] for q in range(nf)]
        lower, upper = [], []
        for c in range(ncell):
            lo, up = [], []
            for q in range(nf):
                half = 0.5 * minmod(diff[q][c], diff[q][idx(c, ax, 1)])
                lo.append(V[c][q] - half)
                up.append(V[c][q] + half)
            lower.append(lo)
            upper.append(up)
        # one flux per face: the face below cell c joins upper(c - 1) and lower(c)
        flux = [hllc(d, g, ax, upper[idx(c, ax, -1)], lower[c]) for c in range(ncell)]
        for c in range(ncell):
            up = idx(c, ax, 1)
            for q in range(nf):
                term = coefs[ax] * (flux[c][q] - flux[up][q])
                acc[q][c] = term if acc[q][c] is None else acc[q][c] + term
    return [[Ubase[q][c] + acc[q][c] for c in range(ncell)] for q in range(nf)]


def cfl_term(d: int, g: Gas, inv_dx: list, u: list) -> F:
    v = prim_of_cons(d, g, u)
    c = fsqrt(g.gamma * v[d + 1] / v[0])
    q = (F(abs(v[1].v)) + c) * inv_dx[0]
    for a in range(1, d):
        q = q + (F(abs(v[1 + a].v)) + c) * inv_dx[a]
    return q


def count_step(d: int, n: tuple, gamma: float, U: np.ndarray, dt: float) -> dict:
    """Operations of one midpoint step (dt given) plus the CFL term of its result, on a
    periodic mesh with cell sizes 1/n_a.  Returns per-cell-update counts by kind and the
    new state (for checking the counted arithmetic against the oracle)."""
    global _C
    _C = Counter()
    g = Gas(gamma)
    n3 = tuple(n) + (1,) * (3 - len(n))
    nf = d + 2
    ncell = n3[0] * n3[1] * n3[2]
    U0 = [[F(x) for x in np.asarray(U[q], dtype=np.float64).ravel()] for q in range(nf)]
    dx = [1.0 / n3[a] for a in range(d)]
    U1 = stage(d, g, n3, U0, U0, [0.5 * dt / dx[a] for a in range(d)])
    U2 = stage(d, g, n3, U1, U0, [dt / dx[a] for a in range(d)])
    for c in range(ncell):
        cfl_term(d, g, [1.0 / x for x in dx], [U2[q][c] for q in range(nf)])
    out = np.array([[x.v for x in U2[q]] for q in range(nf)]).reshape(np.asarray(U).shape)
    per = {k: getattr(_C, k) / ncell for k in ("add", "mul", "div", "sqrt")}
    per["total"] = _C.total / ncell
    return {"per_cell_update": per, "state": out}


def closed_form(d: int) -> dict:
    """Operations per cell-update when every face takes the HLLC star branch (the subsonic
    case), by component; the counting run gives the same on such inputs."""
    nf = d + 2
    vofu = 3 * d + 3                       # 1/rho; d products; v.m (2d - 1); *1/2, -, *(gamma-1)
    recon = d * nf * (1 + 3)               # per axis and primitive: a face difference, half, y -+ half
    side_flux_state = d + (2 * d + 3) + (d + 3)   # momenta, E, flux
    star = d + 9                           # S_K - S*, the factor, d momenta, 7 for the energy
    hllc_star = 6 + 4 + 11 + side_flux_state + star + 3 * nf
    addflux = 3 * d * nf
    stage_ops = vofu + recon + d * hllc_star + addflux
    cfl = vofu + 3 + 2 * d + (d - 1)
    return {"vofu": vofu, "recon_per_cell": recon, "hllc_star_per_face": hllc_star, "addflux": addflux,
            "stage": stage_ops, "cfl": cfl, "total": 2 * stage_ops + cfl}

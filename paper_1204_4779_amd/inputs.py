"""Seeded synthetic initial conditions (shared by the tests, the benchmark and the oracle runs).

This module holds none of the solver's arithmetic.  It defines inputs: a
counter-based random generator and the initial conditions of the workloads,
stated in primitive variables (rho, v, p) and handed out as conserved state
arrays via the ideal-gas definition of the conserved variables
(m = rho v, E = p/(gamma-1) + rho |v|^2 / 2), which is how every initial
condition in the paper is specified.

Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based hash:
value(seed, stream, k) = mix(key(seed, stream) + (k+1) * GOLDEN), with
mix the SplitMix64 finaliser.  Uniforms take the top 53 bits; Gaussians use
Box-Muller on two independent streams.

Arrays: numpy float64 of shape (d+2, nz, ny, nx) (x fastest; leading
dimensions dropped for d < 3), fields rho, m_0..m_{d-1}, E.  Cell centres are
at (i + 1/2)/N on the unit interval along each axis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k = _mix(np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + GOLDEN], dtype=np.uint64))
        k = _mix(k + np.uint64(stream & 0xFFFFFFFFFFFFFFFF) * GOLDEN + GOLDEN)
    return k[0]


def raw64(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Counter values k = start .. start+count-1 of one stream."""
    k = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(_key(seed, stream) + (k + np.uint64(1)) * GOLDEN)


def uniform(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """Uniforms in [0, 1) from the top 53 bits."""
    return (raw64(seed, stream, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """Standard normals: Box-Muller on streams 2*stream (radius) and 2*stream+1 (angle)."""
    u1 = 1.0 - uniform(seed, 2 * stream, count, start)  # (0, 1]
    u2 = uniform(seed, 2 * stream + 1, count, start)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# ----------------------------------------------------------------------------------------
# primitive -> conserved (definition of the conserved variables; used only to state inputs)
# ----------------------------------------------------------------------------------------

def conserved(gamma: float, rho: np.ndarray, vel: list, p: np.ndarray) -> np.ndarray:
    d = len(vel)
    out = np.empty((d + 2,) + rho.shape, dtype=np.float64)
    out[0] = rho
    kin = np.zeros_like(rho)
    for a in range(d):
        out[1 + a] = rho * vel[a]
        kin += vel[a] * vel[a]
    out[d + 1] = p / (gamma - 1.0) + 0.5 * rho * kin
    return out


def centres(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


@dataclass(frozen=True)
class Problem:
    """A named initial condition on one mesh."""
    name: str
    ndim: int
    n: tuple          # (nx, ny, nz) with 1 for unused axes
    gamma: float
    bc: tuple         # per axis: 0 periodic, 1 outflow
    U: np.ndarray     # conserved state, float64


# ----------------------------------------------------------------------------------------
# the paper's validation problems ("Tuning Experiments", convergence tests)
# ----------------------------------------------------------------------------------------

def sod_1d(n: int = 1024, gamma: float = 1.4) -> Problem:
    """Sod's shock tube: (rho, u, p) = (1, 0, 1) for x < 0.5, (0.125, 0, 0.1) otherwise; outflow."""
    x = centres(n)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    u = np.zeros(n)
    return Problem("sod", 1, (n, 1, 1), gamma, (1, 1, 1), conserved(gamma, rho, [u], p))


def entropy_wave_1d(n: int, gamma: float = 1.4) -> Problem:
    """rho = 2 + sin(2 pi x), v = 1, p = 1, periodic: translates with unit speed."""
    x = centres(n)
    rho = 2.0 + np.sin(2.0 * math.pi * x)
    return Problem("entropy", 1, (n, 1, 1), gamma, (0, 0, 0),
                   conserved(gamma, rho, [np.ones(n)], np.ones(n)))


def sound_wave_1d(n: int, gamma: float = 1.4, amp: float = 1e-5) -> Problem:
    """rho = gamma (1 + A s), v = A s, p = 1 + gamma A s with s = sin(2 pi x): unit sound speed."""
    x = centres(n)
    s = np.sin(2.0 * math.pi * x)
    rho = gamma * (1.0 + amp * s)
    v = amp * s
    p = 1.0 + gamma * amp * s
    return Problem("sound", 1, (n, 1, 1), gamma, (0, 0, 0), conserved(gamma, rho, [v], p))


# ----------------------------------------------------------------------------------------
# benchmark workloads
# ----------------------------------------------------------------------------------------

def kelvin_helmholtz_2d(n: int = 2048, seed: int = 1204, gamma: float = 1.4) -> Problem:
    """Periodic shear layer: rho = 2, v_x = +0.5 for 0.25 <= y < 0.75, else rho = 1,
    v_x = -0.5; p = 2.5; v_y = 0.01 (2u - 1), u uniform per cell from `seed`."""
    y = centres(n)[:, None] * np.ones((1, n))
    mid = (y >= 0.25) & (y < 0.75)
    rho = np.where(mid, 2.0, 1.0)
    vx = np.where(mid, 0.5, -0.5)
    vy = 0.01 * (2.0 * uniform(seed, 0, n * n).reshape(n, n) - 1.0)
    p = np.full((n, n), 2.5)
    return Problem("kh", 2, (n, n, 1), gamma, (0, 0, 0), conserved(gamma, rho, [vx, vy], p))


def turbulent_box_3d(n: int = 256, seed: int = 4779, gamma: float = 5.0 / 3.0,
                     z_range: tuple | None = None) -> Problem:
    """Periodic box: rho = exp(0.5 g0) (lognormal, sigma 0.5), v_a = 0.3 c0 g_{a+1} with
    c0 = sqrt(gamma * 1 / 1) the sound speed of the unit state, p = 1.  g_* are independent
    standard normals per cell.  `z_range=(z0, z1)` generates only those z-planes (same values
    as the full box)."""
    z0, z1 = (0, n) if z_range is None else z_range
    nz = z1 - z0
    count = nz * n * n
    start = z0 * n * n
    shape = (nz, n, n)
    c0 = math.sqrt(gamma)
    rho = np.exp(0.5 * gaussian(seed, 0, count, start)).reshape(shape)
    vel = [0.3 * c0 * gaussian(seed, 1 + a, count, start).reshape(shape) for a in range(3)]
    p = np.ones(shape)
    return Problem("box3d", 3, (n, n, nz), gamma, (0, 0, 0), conserved(gamma, rho, vel, p))


def batch_sizes(count: int = 512, seed: int = 12044779, nmin: int = 64, nmax: int = 512) -> list:
    """Square mesh sizes N_k = round(nmin * (nmax/nmin)^u_k): log-uniform cell counts."""
    u = uniform(seed, 0, count)
    return [int(round(nmin * (nmax / nmin) ** float(uk))) for uk in u]


def blob_2d(n: int, seed: int, k: int, gamma: float = 1.4) -> Problem:
    """Gaussian blob of density and pressure on rho = p = 1, v = 0 (periodic), parameters of
    mesh k drawn from `seed`: centre ~ U[0,1)^2, width w ~ U[0.05, 0.15], amplitudes
    A_rho, A_p ~ U[0.5, 2]; r is the periodic minimum-image distance to the centre."""
    par = np.array([uniform(seed, 1 + j, 1, start=k)[0] for j in range(5)])
    cx, cy = par[0], par[1]
    w = 0.05 + 0.10 * par[2]
    arho = 0.5 + 1.5 * par[3]
    ap = 0.5 + 1.5 * par[4]
    x = centres(n)[None, :]
    y = centres(n)[:, None]
    dxp = np.abs(x - cx)
    dyp = np.abs(y - cy)
    dxp = np.minimum(dxp, 1.0 - dxp)
    dyp = np.minimum(dyp, 1.0 - dyp)
    r2 = dxp * dxp + dyp * dyp
    g = np.exp(-r2 / (2.0 * w * w))
    rho = 1.0 + arho * g
    p = 1.0 + ap * g
    z = np.zeros((n, n))
    return Problem(f"blob{k}", 2, (n, n, 1), gamma, (0, 0, 0), conserved(gamma, rho, [z, z], p))


def blob_batch(count: int = 512, seed: int = 12044779, nmin: int = 64, nmax: int = 512) -> list:
    return [blob_2d(nk, seed, k) for k, nk in enumerate(batch_sizes(count, seed, nmin, nmax))]


# ----------------------------------------------------------------------------------------
# generic states for parity tests
# ----------------------------------------------------------------------------------------

def random_state(ndim: int, n: tuple, seed: int, gamma: float = 1.4, bc=(0, 0, 0),
                 rough: bool = False) -> Problem:
    """Random per-cell states.  smooth-ish (rough=False): rho, p in [0.5, 1.5], |v| <= 0.5.
    rough=True: rho, p log-uniform in [0.1, 10], v uniform in [-3, 3] — jumps of every kind,
    including supersonic faces."""
    n3 = tuple(n) + (1,) * (3 - len(n))
    shape = tuple(reversed(n3[:ndim]))
    count = n3[0] * n3[1] * n3[2]
    draws = [uniform(seed, j, count).reshape(shape) for j in range(ndim + 2)]
    if rough:
        rho = 10.0 ** (2.0 * draws[0] - 1.0)
        p = 10.0 ** (2.0 * draws[ndim + 1] - 1.0)
        vel = [6.0 * draws[1 + a] - 3.0 for a in range(ndim)]
    else:
        rho = 0.5 + draws[0]
        p = 0.5 + draws[ndim + 1]
        vel = [draws[1 + a] - 0.5 for a in range(ndim)]
    return Problem("random", ndim, n3, gamma, tuple(bc) + (0,) * (3 - len(bc)),
                   conserved(gamma, rho, vel, p))


def uniform_flow(ndim: int, n: tuple, gamma: float = 1.4, rho: float = 1.3,
                 vel=(0.7, -0.4, 0.25), p: float = 0.9, bc=(0, 0, 0)) -> Problem:
    n3 = tuple(n) + (1,) * (3 - len(n))
    shape = tuple(reversed(n3[:ndim]))
    r = np.full(shape, rho)
    v = [np.full(shape, vel[a]) for a in range(ndim)]
    return Problem("uniform", ndim, n3, gamma, tuple(bc) + (0,) * (3 - len(bc)),
                   conserved(gamma, r, v, np.full(shape, p)))


def cold_stirred_2d(n: tuple, seed: int, amp: float, p0: float = 1e-3, gamma: float = 1.4,
                    bc=(0, 0, 0)) -> Problem:
    """A cold, randomly stirred patch: rho = exp(0.3 g0), v_a = amp g_{a+1} exp(-r^2 / 0.01)
    with r the distance to the mesh centre (0.5, 0.5), p = p0 everywhere.  With a small p0
    the stirring's kinetic energy dwarfs the internal energy, so for some seeds and
    amplitudes the scheme reaches a non-physical state (p <= 0) after a few steps: the
    input of the failure-handling tests."""
    nx, ny = n[0], n[1]
    count = nx * ny
    shape = (ny, nx)
    x = centres(nx)[None, :]
    y = centres(ny)[:, None]
    w = np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / 0.01)
    rho = np.exp(0.3 * gaussian(seed, 0, count).reshape(shape))
    vel = [amp * gaussian(seed, 1 + a, count).reshape(shape) * w for a in range(2)]
    p = np.full(shape, float(p0))
    return Problem("cold_stirred", 2, (nx, ny, 1), gamma, tuple(bc) + (0,) * (3 - len(bc)),
                   conserved(gamma, rho, vel, p))


def cold_stirred_1d(n: int, seed: int, amp: float, p0: float = 1e-3, gamma: float = 1.4, bc: int = 0) -> Problem:
    """The 1D line of `cold_stirred_2d`: rho = exp(0.3 g0), v = amp g1 exp(-(x - 0.5)^2 / 0.01),
    p = p0."""
    x = centres(n)
    w = np.exp(-((x - 0.5) ** 2) / 0.01)
    rho = np.exp(0.3 * gaussian(seed, 0, n))
    vel = [amp * gaussian(seed, 1, n) * w]
    p = np.full(n, float(p0))
    return Problem("cold_stirred", 1, (n, 1, 1), gamma, (bc, 0, 0), conserved(gamma, rho, vel, p))


def cold_stirred_3d(n: tuple, seed: int, amp: float, p0: float = 1e-3, width: float = 0.04,
                    gamma: float = 1.4) -> Problem:
    """The periodic box analogue of `cold_stirred_2d`: rho = exp(0.3 g0),
    v_a = amp g_{a+1} exp(-r^2 / width) with r the distance to the box centre, p = p0."""
    nx, ny, nz = n
    x = centres(nx)[None, None, :]
    y = centres(ny)[None, :, None]
    z = centres(nz)[:, None, None]
    w = np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / width)
    shape = (nz, ny, nx)
    count = nx * ny * nz
    rho = np.exp(0.3 * gaussian(seed, 0, count).reshape(shape))
    vel = [amp * gaussian(seed, 1 + a, count).reshape(shape) * w for a in range(3)]
    p = np.full(shape, float(p0))
    return Problem("cold_stirred", 3, (nx, ny, nz), gamma, (0, 0, 0), conserved(gamma, rho, vel, p))


# ----------------------------------------------------------------------------------------
# the same generator in torch (any device): the large 3D boxes are generated where they
# are used instead of on the host.  The uniforms are bit-identical to the numpy ones; the
# Box-Muller transcendental functions of the device may differ from the host's libm in
# the last bit of an FP64 value.
# ----------------------------------------------------------------------------------------

def _srl_t(z, k: int):
    """Logical right shift of uint64 bit patterns held in an int64 tensor."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _signed(v: int) -> int:
    v &= 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >= (1 << 63) else v


def _mix_t(z):
    z = (z ^ _srl_t(z, 30)) * _signed(int(_M1))
    z = (z ^ _srl_t(z, 27)) * _signed(int(_M2))
    return z ^ _srl_t(z, 31)


def uniform_torch(seed: int, stream: int, count: int, start: int = 0, device="cpu"):
    """`uniform` as a float64 torch tensor on `device` (same values, bit for bit)."""
    import torch
    k = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = _mix_t(k * _signed(int(GOLDEN)) + _signed(int(_key(seed, stream))))
    return _srl_t(z, 11).to(torch.float64) * (2.0 ** -53)


def gaussian_torch(seed: int, stream: int, count: int, start: int = 0, device="cpu"):
    import torch
    u1 = 1.0 - uniform_torch(seed, 2 * stream, count, start, device)
    u2 = uniform_torch(seed, 2 * stream + 1, count, start, device)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


def turbulent_box_3d_torch(n: int = 256, seed: int = 4779, gamma: float = 5.0 / 3.0,
                           z_range: tuple | None = None, device="cpu"):
    """`turbulent_box_3d(...).U` for the planes z_range, as a float64 torch tensor of shape
    (5, nz, n, n) on `device`."""
    import torch
    z0, z1 = (0, n) if z_range is None else z_range
    nz = z1 - z0
    count = nz * n * n
    start = z0 * n * n
    shape = (nz, n, n)
    c0 = math.sqrt(gamma)
    rho = torch.exp(0.5 * gaussian_torch(seed, 0, count, start, device)).reshape(shape)
    out = torch.empty((5,) + shape, dtype=torch.float64, device=device)
    out[0] = rho
    kin = torch.zeros(shape, dtype=torch.float64, device=device)
    for a in range(3):
        v = 0.3 * c0 * gaussian_torch(seed, 1 + a, count, start, device).reshape(shape)
        out[1 + a] = rho * v
        kin += v * v
    out[4] = 1.0 / (gamma - 1.0) + 0.5 * rho * kin
    return out

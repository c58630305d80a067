"""Helpers shared by the GPU tests: run the HIP path through the C ABI and compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1204_4779_amd import binding as pb

# tolerances (relative, per field normwise and pointwise for rho and E, one step
# from identical input)
TOL = {"f64": 1e-12, "f32": 1e-5}

VARIANTS = {
    # name: (lds, fuse); "default": the library's own choice for the meshes
    # (resident 1D, register march 2D periodic / 3D, else LDS tiles)
    "direct": dict(lds=0, fuse=0),
    "direct_fused": dict(lds=0, fuse=1),
    "lds": dict(lds=1, fuse=0),
    "lds_fused": dict(lds=1, fuse=1),
    "default": None,
}


def default_tile(ndim: int):
    return {1: (64, 1, 1), 2: (16, 8, 1), 3: (8, 4, 4)}[ndim]


def spec_of(pr) -> pb.MeshSpec:
    return pb.MeshSpec(pr.ndim, pr.n, pr.gamma, pr.bc)


def oracle_mesh(pr, dx=None) -> oracle.Mesh:
    return oracle.Mesh(pr.ndim, pr.n, pr.gamma, pr.bc, dx=dx)


def as_input(U: np.ndarray, dtype: str) -> np.ndarray:
    """The FP64 values the GPU actually starts from (FP32 inputs are rounded once)."""
    return U.astype(np.float32).astype(np.float64) if dtype == "f32" else U


def pointwise_err(got: np.ndarray, ref: np.ndarray) -> float:
    """Pointwise relative error of the strictly positive fields, density and
    energy: max over cells of |got - ref| / |ref|, the second half of the
    relative-error reading (normwise per field, and pointwise for rho and E)."""
    worst = 0.0
    for q in (0, ref.shape[0] - 1):
        r = np.abs(ref[q])
        assert np.all(r > 0), "pointwise error needs a strictly positive field"
        worst = max(worst, float(np.max(np.abs(got[q] - ref[q]) / r)))
    return worst


def normwise_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max over fields of max|got - ref| / max|ref| (fields with ref == 0 use absolute error)."""
    worst = 0.0
    for q in range(ref.shape[0]):
        scale = float(np.max(np.abs(ref[q])))
        d = float(np.max(np.abs(got[q] - ref[q])))
        worst = max(worst, d / scale if scale > 0 else d)
    return worst


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """The strict measure: every field normwise against its own maximum, and
    density and energy also pointwise (the larger of the two)."""
    return max(normwise_err(got, ref), pointwise_err(got, ref))


def gpu_solver(specs, dtype, variant=None, states=None):
    s = pb.Solver(specs, dtype)
    if variant is not None:
        s.set_variant(variant)
    if states is not None:
        s.upload(states)
    return s


def gpu_state(s, m=0) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return s.state(m).double().cpu().numpy()


def field_errs(got: np.ndarray, ref: np.ndarray) -> list:
    """Per-field max|got - ref| / max|ref|."""
    out = []
    for q in range(ref.shape[0]):
        scale = float(np.max(np.abs(ref[q])))
        d = float(np.max(np.abs(got[q] - ref[q])))
        out.append(d / scale if scale > 0 else d)
    return out


def state_scaled_err(got: np.ndarray, ref: np.ndarray, gamma: float) -> float:
    """Relative error with each field measured against its own natural scale:
    density and energy against max|rho| and max|E|, each momentum component
    against max rho (|v| + c) (momentum of the fastest signal), so that a
    momentum field that starts at rest is not measured against its own
    vanishing size.  All scales from the reference."""
    d = ref.shape[0] - 2
    rho = ref[0]
    m2 = sum(ref[1 + a] ** 2 for a in range(d))
    vel = np.sqrt(m2) / rho
    p = (gamma - 1.0) * (ref[d + 1] - 0.5 * m2 / rho)
    c = np.sqrt(gamma * np.maximum(p, 0.0) / rho)
    mscale = float(np.max(rho * (vel + c)))
    worst = 0.0
    for q in range(ref.shape[0]):
        scale = mscale if 1 <= q <= d else float(np.max(np.abs(ref[q])))
        worst = max(worst, float(np.max(np.abs(got[q] - ref[q]))) / scale)
    return worst


def state_err(got: np.ndarray, ref: np.ndarray, gamma: float) -> float:
    """The measure for momenta that start at rest or as a small perturbation:
    the state-scaled error, and density and energy also pointwise (the larger
    of the two)."""
    return max(state_scaled_err(got, ref, gamma), pointwise_err(got, ref))


def strict_err(got: np.ndarray, ref: np.ndarray, gamma: float, zero: float = 1e-10) -> float:
    """The strict measure for fields that may vanish in exact arithmetic: every
    field normwise against its own maximum, except a momentum component whose
    own maximum is below `zero` times max rho (|v| + c) (a component that is
    zero in exact arithmetic and holds only rounding, such as the transverse
    momentum of a wave along an axis), which has no scale of its own and is
    measured against max rho (|v| + c); density and energy also pointwise."""
    d = ref.shape[0] - 2
    rho = ref[0]
    m2 = sum(ref[1 + a] ** 2 for a in range(d))
    c = np.sqrt(gamma * np.maximum((gamma - 1.0) * (ref[d + 1] - 0.5 * m2 / rho), 0.0) / rho)
    mscale = float(np.max(np.sqrt(m2) + rho * c))
    worst = pointwise_err(got, ref)
    for q in range(ref.shape[0]):
        own = float(np.max(np.abs(ref[q])))
        scale = mscale if (1 <= q <= d and own < zero * mscale) else own
        worst = max(worst, float(np.max(np.abs(got[q] - ref[q]))) / scale)
    return worst


def measures(got: np.ndarray, ref: np.ndarray, gamma: float) -> dict:
    """Every measure, for the logs: strict per field, pointwise rho and E, state-scaled."""
    return {"per_field": [float(f"{e:.3e}") for e in field_errs(got, ref)],
            "pointwise_rho_E": float(f"{pointwise_err(got, ref):.3e}"),
            "state_scaled": float(f"{state_scaled_err(got, ref, gamma):.3e}")}

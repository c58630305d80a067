"""Helpers shared by the GPU tests: run the HIP path through the C ABI and compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1204_4779_amd import binding as pb

# tolerances (normwise relative, per field, one step from identical input)
TOL = {"f64": 1e-12, "f32": 1e-5}

VARIANTS = {
    # name: (lds, fuse)
    "direct": dict(lds=0, fuse=0),
    "direct_fused": dict(lds=0, fuse=1),
    "lds": dict(lds=1, fuse=0),
    "lds_fused": dict(lds=1, fuse=1),
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


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max over fields of max|got - ref| / max|ref| (fields with ref == 0 use absolute error)."""
    worst = 0.0
    for q in range(ref.shape[0]):
        scale = float(np.max(np.abs(ref[q])))
        d = float(np.max(np.abs(got[q] - ref[q])))
        worst = max(worst, d / scale if scale > 0 else d)
    return worst


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

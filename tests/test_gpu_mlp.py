"""The tuner's MLP kernels (paraiso_mlp_*) against the FP64 reference, and the variant
space's static validity against the runtime's own checks."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1204_4779_amd import binding as pb
from paper_1204_4779_amd.tuner import search
from paper_1204_4779_amd.tuner import space as sp

pytestmark = pytest.mark.gpu

IN, H = 16, 64


def _setup(B, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    n, ws = pb.paraiso_mlp_sizes(IN, H, B)
    assert n == omlp.n_params(IN, H)
    p = (rng.normal(scale=0.3, size=n)).astype(np.float32)
    X = rng.normal(size=(B, IN)).astype(np.float32)
    T = rng.normal(size=B).astype(np.float32)
    dev = torch.device("cuda", 0)
    d = {k: torch.from_numpy(v).to(dev) for k, v in (("p", p), ("X", X), ("T", T))}
    d["ws"] = torch.empty(ws // 4 + 64, dtype=torch.float32, device=dev)
    d["ws_bytes"] = ws
    d["stream"] = torch.cuda.current_stream().cuda_stream
    return p, X, T, n, d


def test_forward_matches_reference():
    import torch
    B = 37
    p, X, T, n, d = _setup(B)
    y = torch.empty(B, dtype=torch.float32, device="cuda")
    pb.paraiso_mlp_forward(d["X"].data_ptr(), B, IN, H, d["p"].data_ptr(), y.data_ptr(), d["ws"].data_ptr(),
                           d["ws_bytes"], d["stream"])
    got = y.cpu().numpy().astype(np.float64)
    ref, _ = omlp.forward(X.astype(np.float64), p.astype(np.float64), IN, H)
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5 * np.max(np.abs(ref)))


def test_gradient_matches_reference_and_is_deterministic():
    import torch
    B = 53
    p, X, T, n, d = _setup(B, seed=1)
    g1 = torch.empty(n, dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for g in (g1, g2):
        pb.paraiso_mlp_loss_grad(d["X"].data_ptr(), d["T"].data_ptr(), B, IN, H, d["p"].data_ptr(), g.data_ptr(),
                                 loss.data_ptr(), d["ws"].data_ptr(), d["ws_bytes"], d["stream"])
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    ref_loss, ref_g = omlp.loss_grad(X.astype(np.float64), T.astype(np.float64), p.astype(np.float64), IN, H)
    assert abs(loss.item() - ref_loss) <= 1e-5 * ref_loss
    got = g1.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref_g)) <= 1e-5 * np.max(np.abs(ref_g))


def test_adam_matches_reference():
    import torch
    B = 20
    p, X, T, n, d = _setup(B, seed=2)
    g = torch.empty(n, dtype=torch.float32, device="cuda")
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    rp, rm, rv = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        pb.paraiso_mlp_loss_grad(d["X"].data_ptr(), d["T"].data_ptr(), B, IN, H, d["p"].data_ptr(), g.data_ptr(),
                                 0, d["ws"].data_ptr(), d["ws_bytes"], d["stream"])
        torch.cuda.synchronize()
        gg = g.cpu().numpy().astype(np.float64)
        pb.paraiso_mlp_adam(d["p"].data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), n, 1e-2, 0.9, 0.999,
                            1e-8, step, d["stream"])
        rp, rm, rv = omlp.adam(rp, gg, rm, rv, 1e-2, 0.9, 0.999, 1e-8, step)
        torch.cuda.synchronize()
        got = d["p"].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, rp, rtol=1e-5, atol=1e-6)
        rp = got  # continue from the device's rounding


def test_training_fits_a_smooth_target():
    from paper_1204_4779_amd.tuner.model import CostModel
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, size=(200, 6))
    y = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 3] ** 2
    m = CostModel(6, 64, seed=0, max_batch=256)
    first = m.fit(X, y, epochs=1)
    last = m.fit(X, y, epochs=800)
    assert last < 0.1 * first
    pred = m.predict(X)
    assert np.corrcoef(pred, y)[0, 1] > 0.95


@pytest.mark.parametrize("ndim,dtype", [(3, "f32"), (2, "f32"), (2, "f64")])
def test_static_validity_agrees_with_runtime(ndim, dtype):
    from paper_1204_4779_amd import inputs
    n = (24,) * ndim
    pr = inputs.random_state(ndim, n, seed=0)
    s = pb.Solver(pb.MeshSpec(ndim, n, pr.gamma, (0,) * 3), dtype)
    esize = 4 if dtype == "f32" else 8
    for v in sp.enumerate_space(ndim):
        want = sp.statically_valid(v, ndim, esize)
        try:
            s.set_variant(v)
            got = True
        except pb.ParaisoError as e:
            assert e.code == pb.ERR_UNSUPPORTED
            got = False
        assert got == want, v

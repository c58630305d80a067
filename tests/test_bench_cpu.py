"""bench.py's contract pieces that need no GPU: the single-GPU guard, the
roofline bookkeeping and the counted work per cell-update."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_bytes_and_flops():
    assert bench.bytes_per_cell_update(2, 4) == 32
    assert bench.bytes_per_cell_update(3, 8) == 80
    # the non-packed FP32 ALU roof: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
    assert abs(bench.ALU_PEAK_NONPACKED_TFLOPS["f32"] - 256 * 4 * 16 * 2 * 2.4e9 / 1e12) < 0.1
    assert bench.ALU_PEAK_TFLOPS["f32"] == 157.3


def test_flop_count_is_the_methods_own_count():
    # the per-cell figures bench.py uses are what the counting run of the method reports
    # for one step (+ CFL) of the KH workload, and the closed form by component
    import oracle
    from oracle import method_flops as mf
    from paper_1204_4779_amd import inputs
    pr = inputs.kelvin_helmholtz_2d(32)
    m = oracle.Mesh(2, pr.n, pr.gamma, pr.bc)
    r = mf.count_step(2, (32, 32), pr.gamma, pr.U, oracle.cfl_dt(m, pr.U, 0.5))
    assert r["per_cell_update"]["total"] == bench.FLOPS_PER_CELL_UPDATE[2]
    for d in (1, 2, 3):
        assert mf.closed_form(d)["total"] == bench.FLOPS_PER_CELL_UPDATE[d]


def test_oracle_code_count_is_an_upper_bound():
    # the counting build of the oracle counts its own (recomputing) code: the figure
    # bench.py reports beside the method's count
    import oracle
    from paper_1204_4779_amd import inputs
    pr = inputs.kelvin_helmholtz_2d(256)
    counts = oracle.count_ops(oracle.Mesh(2, pr.n, pr.gamma, pr.bc), pr.U, 1e-4)
    per_cell = counts["add"] + counts["mul"] + counts["div"] + counts["sqrt"]
    assert abs(per_cell - bench.FLOPS_ORACLE_CODE[2]) / bench.FLOPS_ORACLE_CODE[2] < 2e-3
    assert per_cell > bench.FLOPS_PER_CELL_UPDATE[2]


def test_kernel_name_follows_the_variant():
    assert bench.kernel_name(dict(tile=(64, 20), lds=2, fuse=1, waves_per_eu=0)) == "k_march2d<float,0,true>"
    assert bench.kernel_name(dict(tile=(64, 16), lds=2, fuse=0, waves_per_eu=4)) == "k_march2d<float,4,false>"
    assert bench.kernel_name(dict(tile=(32, 16), lds=1, fuse=1)) == "k_fused_lds<float,2,0>"


def test_traffic_constant_is_the_one_its_profile_records():
    # bench.py reports the measured HBM bytes only for the kernel sources and
    # variant they were counted on; the committed profile of that kernel must
    # name the same sources and bytes
    text = open(os.path.join(ROOT, "profiles", "k_march2d_f32_kh2048.md")).read()
    assert f"`{bench.TRAFFIC['sources']}`" in text
    assert f"Measured {bench.TRAFFIC['bytes_per_launch'] / 1e6:.1f} MB per launch" in text
    v = bench.TRAFFIC["variant"]
    assert f"tile ({v['tile'][0]}, {v['tile'][1]})" in text and f"{v['threads']} threads" in text


def test_counted_method_is_the_scheme():
    # the code the method's operations are counted on computes the oracle's step (rough
    # states reach every HLLC branch), so the count is of the scheme and nothing else
    import numpy as np
    import oracle
    from oracle import method_flops as mf
    from paper_1204_4779_amd import inputs
    for d, n in ((1, (40,)), (2, (12, 10)), (3, (6, 5, 4))):
        for rough in (False, True):
            pr = inputs.random_state(d, n, seed=40 + d, rough=rough)
            m = oracle.Mesh(d, pr.n, pr.gamma, pr.bc)
            dt = oracle.cfl_dt(m, pr.U, 0.5)
            r = mf.count_step(d, n, pr.gamma, pr.U, dt)
            ref = oracle.step(m, pr.U, dt)
            for q in range(d + 2):
                assert np.max(np.abs(r["state"][q] - ref[q])) <= 1e-13 * np.max(np.abs(ref[q]))
            # supersonic faces take fewer operations than the star branch
            assert r["per_cell_update"]["total"] <= mf.closed_form(d)["total"]
            if not rough:
                assert r["per_cell_update"]["total"] == mf.closed_form(d)["total"]

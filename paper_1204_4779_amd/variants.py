"""Kernel variants chosen per workload (tile, LDS staging, stage fusion, occupancy hint).

`TUNED` holds the best variant measured for each workload and precision by the
tuner (exhaustive search over the variant space on an MI355X); `UNTUNED` is the
per-cell, unfused, unstaged kernel — every cell recomputes its own face fluxes —
which plays the role of the paper's untuned baseline.
"""

UNTUNED_2D = dict(tile=(64, 4), lds=0, fuse=0, waves_per_eu=0, threads=256)
UNTUNED_3D = dict(tile=(16, 4, 4), lds=0, fuse=0, waves_per_eu=0, threads=256)

TUNED = {
    # register march, fused RK, stage-1 rows shared between the 4 waves of a
    # block.  The rows per wave come from a sweep of rows x threads x
    # occupancy hint on top of the exhaustive search (whose tile axis has
    # 8/16/32/64 only).  FP32: <= 128 VGPRs, 4 waves per SIMD, and 37 strips x
    # 27 row blocks = 999 blocks of 4 waves, all resident at once; FP64: 2
    # waves per SIMD, 37 strips x 13 row blocks of 158 rows = 481 blocks of 4
    # waves (36.1-36.8 G against 35.3-35.7 G for 2 waves of 40 rows).
    ("kh2048", "f32"): dict(tile=(64, 20), lds=2, fuse=1, waves_per_eu=0, threads=256),
    ("kh2048", "f64"): dict(tile=(64, 40), lds=2, fuse=1, waves_per_eu=0, threads=256),
    # 3D register march, one stage per launch: 60 columns x 4 rows per block,
    # 64-plane chunks, VGPRs capped at 168 (3 waves per SIMD)
    ("box256", "f32"): dict(tile=(64, 4, 64), lds=2, fuse=0, waves_per_eu=3),
    ("box512", "f32"): dict(tile=(64, 4, 64), lds=2, fuse=0, waves_per_eu=3),
    # one launch per step over every (mesh, tile) item, one block per item on
    # a plain grid mapped onto the XCDs; 32 rows per wave from a rows sweep
    # (the persistent queue over the same items: 62.2-62.4 against 64.5-64.9 G)
    ("batch512", "f32"): dict(tile=(64, 32), lds=2, fuse=1, waves_per_eu=0, threads=256, persistent=0),
    # the whole advance in one launch, one workgroup holding the 1024 cells
    ("sod1024", "f64"): dict(tile=(1024,), lds=3, fuse=1),
    # convergence tests with analytic boundaries, N <= 1024: the one-stage
    # register march reading ghost arrays, from a rows x threads x hint sweep
    # at 1024^2 (the unfused LDS tile, which evaluates the exact solution
    # in its edge tiles, is 2.1x / 1.8x slower); FP64 with the 3-waves hint
    # (168 VGPRs instead of 173: 3 waves per SIMD, 16.2 against 15.7 G for the
    # best uncapped variant, 12 rows)
    ("convergence", "f32"): dict(tile=(64, 8), lds=2, fuse=0, waves_per_eu=0, threads=256),
    ("convergence", "f64"): dict(tile=(64, 8), lds=2, fuse=0, waves_per_eu=3, threads=256),
}


# the fused 3D register march (both stages in one launch, U1 on chip):
# 12 stage-1 rows per block of 12 waves (8 output rows), 64-plane chunks
FUSED_3D = dict(tile=(64, 12, 64), lds=2, fuse=1, waves_per_eu=0)
# the one-stage 3D register march (two launches per step, U1 in the workspace)
ONE_STAGE_3D = dict(tile=(64, 4, 64), lds=2, fuse=0, waves_per_eu=3)


def tuned(workload: str, dtype: str) -> dict:
    return dict(TUNED[(workload, dtype)])

"""The C ABI without a GPU: the library loads, exports what include/paraiso.h declares,
and its host-side validation returns the documented status codes."""
import ctypes
import os
import re

import pytest

from paper_1204_4779_amd import binding as pb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paraiso.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pb.LIB_PATH):
        from paper_1204_4779_amd import build
        build.build(verbose=False)
    return pb.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(paraiso_[a-z_]+)\s*\(", text, re.M)))


def test_header_declares_the_binding_names():
    assert set(declared_functions()) == set(pb.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _mesh(ndim=2, n=(8, 8, 1), dtype=pb.F32, gamma=1.4, bc=(0, 0, 0), base=0x10000, dx=None, order=0):
    m = pb.paraiso_mesh()
    m.ndim, m.dtype, m.gamma, m.order = ndim, dtype, gamma, order
    for a in range(3):
        m.n[a] = n[a]
        m.dx[a] = (dx[a] if dx else 1.0 / max(n[a], 1))
        m.bc[a] = bc[a]
    cells = max(n[0] * n[1] * n[2], 1)
    esz = 4 if dtype == pb.F32 else 8
    p = base
    for b in range(2):
        for q in range(min(max(ndim, 1) + 2, 5)):
            m.state[b][q] = p
            p += ((cells * esz + 255) // 256) * 256
    return m


def test_workspace_bytes_valid(lib):
    assert pb.paraiso_workspace_bytes([_mesh()]) > 8 * 8 * 4 * 4
    assert pb.paraiso_workspace_bytes([_mesh(3, (4, 5, 6), pb.F64), _mesh(3, (7, 2, 3), pb.F64)]) > 0


@pytest.mark.parametrize("bad", [
    dict(ndim=0), dict(ndim=4), dict(gamma=1.0), dict(gamma=float("nan")), dict(n=(0, 8, 1)),
    dict(ndim=2, n=(8, 8, 2)), dict(bc=(3, 0, 0)), dict(bc=(0, -1, 0)), dict(dtype=7), dict(dx=(0.0, 1.0, 1.0)),
    dict(dx=(float("inf"), 1.0, 1.0)), dict(order=3), dict(order=-1),
])
def test_workspace_bytes_rejects_invalid_mesh(lib, bad):
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_workspace_bytes([_mesh(**bad)])
    assert ei.value.code == pb.ERR_INVALID_ARG
    assert lib.paraiso_last_error().decode() != ""


def test_rejects_null_and_overlapping_buffers(lib):
    m = _mesh()
    m.state[1][0] = None
    with pytest.raises(pb.ParaisoError):
        pb.paraiso_workspace_bytes([m])
    m = _mesh()
    m.state[1][2] = m.state[0][1]
    with pytest.raises(pb.ParaisoError):
        pb.paraiso_workspace_bytes([m])
    m = _mesh()
    m.state[0][0] = m.state[0][0] + 4  # misaligned
    with pytest.raises(pb.ParaisoError):
        pb.paraiso_workspace_bytes([m])


def test_rejects_mixed_batch(lib):
    with pytest.raises(pb.ParaisoError):
        pb.paraiso_workspace_bytes([_mesh(), _mesh(ndim=3, n=(4, 4, 4), base=0x900000)])


def test_too_many_cells_unsupported(lib):
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_workspace_bytes([_mesh(3, (2048, 2048, 1024))])
    assert ei.value.code == pb.ERR_UNSUPPORTED


def test_init_argument_errors_before_device_work(lib):
    arr = (pb.paraiso_mesh * 1)(_mesh())
    ctx = ctypes.c_void_p()
    assert lib.paraiso_init(arr, 1, None, 1 << 20, None, ctypes.byref(ctx)) == pb.ERR_INVALID_ARG
    assert lib.paraiso_init(arr, 1, ctypes.c_void_p(0x1001), 1 << 20, None, ctypes.byref(ctx)) == pb.ERR_INVALID_ARG
    assert lib.paraiso_init(arr, 1, ctypes.c_void_p(0x100000), 16, None, ctypes.byref(ctx)) == pb.ERR_WORKSPACE
    assert lib.paraiso_init(arr, 0, ctypes.c_void_p(0x100000), 1 << 20, None, ctypes.byref(ctx)) == pb.ERR_INVALID_ARG
    assert lib.paraiso_destroy(None) == pb.OK


def test_default_variant(lib):
    # 2D periodic: the fused register march; any outflow axis: LDS tiles
    v = pb.paraiso_default_variant([_mesh()])
    assert (v.lds, v.fuse, tuple(v.tile)) == (2, 1, (64, 20, 1)) and v.threads == 256
    v = pb.paraiso_default_variant([_mesh(dtype=pb.F64)])
    assert (v.lds, tuple(v.tile), v.threads) == (2, (64, 40, 1), 256)
    v = pb.paraiso_default_variant([_mesh(), _mesh(bc=(0, 1, 0))])
    assert v.lds == 1 and v.fuse == 1 and v.persistent == 0   # batches: one workgroup per tile
    # 3D: the one-stage register march
    v3 = pb.paraiso_default_variant([_mesh(3, (4, 4, 4))])
    assert (v3.lds, v3.fuse, tuple(v3.tile), v3.waves_per_eu) == (2, 0, (64, 4, 64), 3)
    # 1D: resident while every mesh fits one workgroup's LDS
    assert pb.paraiso_default_variant([_mesh(1, (4096, 1, 1))]).lds == 3
    assert pb.paraiso_default_variant([_mesh(1, (4097, 1, 1))]).lds == 1
    assert pb.paraiso_default_variant([_mesh(1, (3407, 1, 1), pb.F64)]).lds == 3
    assert pb.paraiso_default_variant([_mesh(1, (3408, 1, 1), pb.F64)]).lds == 1
    assert pb.paraiso_default_variant([_mesh(1, (4096, 1, 1))]).threads == 1024
    assert pb.paraiso_default_variant([_mesh(1, (2048, 1, 1))]).threads == 512
    assert pb.paraiso_default_variant([_mesh(1, (2049, 1, 1))]).threads == 1024
    v1 = pb.paraiso_default_variant([_mesh(1, (100, 1, 1)), _mesh(1, (1000, 1, 1))])
    assert (v1.lds, v1.tile[0], v1.persistent) == (3, 1000, 0)
    # the march kernels take 32-bit byte offsets within a row (2D) / plane (3D)
    assert pb.paraiso_default_variant([_mesh(2, (1 << 29, 2, 1))]).lds == 2
    assert pb.paraiso_default_variant([_mesh(2, (1 << 30, 1, 1))]).lds == 1
    assert pb.paraiso_default_variant([_mesh(2, (1 << 29, 2, 1), pb.F64)]).lds == 1
    assert pb.paraiso_default_variant([_mesh(3, (1 << 15, 1 << 14, 1))]).lds == 2
    assert pb.paraiso_default_variant([_mesh(3, (1 << 15, 1 << 15, 1))]).lds == 1
    # any analytic axis: the unfused LDS-tile kernel (ghosts at each stage's own time)
    # (2D: the one-stage register march, which reads ghost arrays)
    for d, n in ((1, (64, 1, 1)), (2, (8, 8, 1)), (3, (4, 4, 4))):
        v = pb.paraiso_default_variant([_mesh(d, n, bc=(pb.ANALYTIC, 0, 0))])
        assert (v.lds, v.fuse) == ((2, 0) if d == 2 else (1, 0)), d
    # the analytic march's ghost arrays take 32-bit offsets: meshes past them get
    # LDS tiles (exact solution in place) and no ghost arrays in the workspace
    fits = _mesh(2, ((1 << 26) - 100, 2, 1), bc=(pb.ANALYTIC, 0, 0))
    big = _mesh(2, (1 << 26, 2, 1), bc=(pb.ANALYTIC, 0, 0))
    assert pb.paraiso_default_variant([fits]).lds == 2
    assert pb.paraiso_default_variant([big]).lds == 1
    ghosts = 2 * 4 * (4 * (2 + 4) + 4 * ((1 << 26) - 100 + 4)) * 4
    assert pb.paraiso_workspace_bytes([fits]) > ghosts
    assert pb.paraiso_workspace_bytes([big]) < pb.paraiso_workspace_bytes([fits])
    v = pb.paraiso_default_variant([_mesh(), _mesh(bc=(0, pb.ANALYTIC, 0))])
    assert (v.lds, v.fuse, v.persistent, tuple(v.tile)) == (2, 0, 0, (64, 8, 1))
    v = pb.paraiso_default_variant([_mesh(dtype=pb.F64, bc=(pb.ANALYTIC,) * 3)])
    assert (tuple(v.tile), v.waves_per_eu) == ((64, 8, 1), 3)   # FP64: capped at 3 waves per SIMD
    # first-order reconstruction: the LDS-tile kernels (fused unless analytic)
    for d, n in ((1, (64, 1, 1)), (2, (8, 8, 1)), (3, (4, 4, 4))):
        v = pb.paraiso_default_variant([_mesh(d, n, order=1)])
        assert v.lds == 1 and v.fuse == (0 if d == 3 else 1), d
        v = pb.paraiso_default_variant([_mesh(d, n, order=1, bc=(pb.ANALYTIC, 0, 0))])
        assert (v.lds, v.fuse) == (1, 0), d
    assert pb.paraiso_default_variant([_mesh(order=2)]).lds == 2


def test_batch_must_share_the_reconstruction_order(lib):
    pb.paraiso_workspace_bytes([_mesh(order=1), _mesh(order=1, base=0x8000000)])
    pb.paraiso_workspace_bytes([_mesh(order=0), _mesh(order=2, base=0x8000000)])
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_workspace_bytes([_mesh(order=1), _mesh(order=2, base=0x8000000)])
    assert ei.value.code == pb.ERR_INVALID_ARG


def test_version(lib):
    assert "gfx950" in pb.paraiso_version()


def test_header_compiles_as_c_and_cpp(tmp_path):
    # the boundary is plain C: the header must stand alone in C99 and C++17
    import shutil
    import subprocess
    inc = os.path.join(ROOT, "include")
    src = tmp_path / "use.c"
    src.write_text('#include "paraiso.h"\nint main(void) { paraiso_variant v; (void)v; return PARAISO_OK; }\n')
    for cc, std in (("gcc", "-std=c99"), ("g++", "-std=c++17")):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not found")
        lang = ["-x", "c++"] if cc == "g++" else []
        r = subprocess.run([cc, std, "-Wall", "-Werror", "-fsyntax-only", "-I", inc] + lang + [str(src)],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_wave_entry_points_validate_before_any_device_work(lib):
    import ctypes
    assert pb.paraiso_wave_workspace_bytes(1) == 256
    assert pb.paraiso_wave_workspace_bytes(10) >= 10 * 64
    with pytest.raises(pb.ParaisoError):
        pb.paraiso_wave_workspace_bytes(0)
    ws = 0x100000          # never touched: every case below fails validation first

    def line(**kw):
        w = pb.paraiso_wave()
        w.n, w.c, w.dx, w.dt, w.f, w.g, w.energy = 64, 1.0, 0.1, 0.05, 0x2000, 0x4000, None
        for k, v in kw.items():
            setattr(w, k, v)
        return w
    bad = [dict(n=2), dict(n=4097), dict(c=-1.0), dict(c=float("nan")), dict(dx=0.0), dict(dt=float("inf")),
           dict(f=None), dict(g=0x4004), dict(energy=0x6001)]
    for kw in bad:
        with pytest.raises(pb.ParaisoError) as ei:
            pb.paraiso_wave_advance([line(**kw)], 10, ws, 256, 0)
        assert ei.value.code == pb.ERR_INVALID_ARG, kw
        assert "line 0" in str(ei.value), kw
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_wave_advance([line()], -1, ws, 256, 0)
    assert ei.value.code == pb.ERR_INVALID_ARG
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_wave_advance([line()], 1, ws + 8, 256, 0)
    assert ei.value.code == pb.ERR_INVALID_ARG
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_wave_advance([line()] * 8, 1, ws, 256, 0)
    assert ei.value.code == pb.ERR_WORKSPACE
    for args in ((ws, 1, 1, 2), (ws, 1, 1, 4097), (ws, 0, 1, 64), (ws, 1, -1, 64), (ws + 8, 1, 1, 64)):
        with pytest.raises(pb.ParaisoError) as ei:
            pb.paraiso_wave_run(*args, 0)
        assert ei.value.code == pb.ERR_INVALID_ARG, args


def test_static_cfl_host_validation(lib):
    """paraiso_cfl_dt_static rejects its arguments before touching the device."""
    m = _mesh()
    for meshes, buf, cfl, code in (([m] * (pb.STATIC_MESHES + 1), 0, 0.5, pb.ERR_UNSUPPORTED),
                                   ([m], 2, 0.5, pb.ERR_INVALID_ARG), ([m], 0, 0.0, pb.ERR_INVALID_ARG),
                                   ([m], 0, 1.5, pb.ERR_INVALID_ARG), ([m, _mesh(dtype=pb.F64)], 0, 0.5, pb.ERR_INVALID_ARG),
                                   ([_mesh(ndim=4)], 0, 0.5, pb.ERR_INVALID_ARG), ([_mesh(gamma=0.5)], 0, 0.5, pb.ERR_INVALID_ARG)):
        with pytest.raises(pb.ParaisoError) as ei:
            pb.paraiso_cfl_dt_static(meshes, buf, cfl, 0)
        assert ei.value.code == code
        assert "cfl_dt_static" in lib.paraiso_last_error().decode()
    with pytest.raises(pb.ParaisoError) as ei:
        pb.paraiso_cfl_dt_static([], 0, 0.5, 0)
    assert ei.value.code == pb.ERR_INVALID_ARG

"""ctypes binding of libparaiso.so (include/paraiso.h).

Argument marshalling only: every step of the solver runs in the HIP library.
The functions below have the names of the C entry points and raise
`ParaisoError` on a non-zero status.  `Solver` is a convenience wrapper that
allocates the state buffers and the workspace as torch tensors on the
current device and passes torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libparaiso.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED = -2
ERR_HIP = -3
ERR_NONFINITE = -4
ERR_WORKSPACE = -5
STATIC_MESHES = 64   # PARAISO_STATIC_MESHES: capacity of paraiso_cfl_dt_static

PERIODIC = 0
OUTFLOW = 1
ANALYTIC = 2
ENTROPY_WAVE = 1
SOUND_WAVE = 2
SHOCK_TUBE = 3
F32 = 0
F64 = 1

EXPORTS = ("paraiso_workspace_bytes", "paraiso_init", "paraiso_set_variant", "paraiso_get_variant",
           "paraiso_default_variant", "paraiso_cfl_dt", "paraiso_step", "paraiso_advance",
           "paraiso_current", "paraiso_totals", "paraiso_destroy", "paraiso_last_error",
           "paraiso_version", "paraiso_set_analytic", "paraiso_exact_state", "paraiso_set_time", "paraiso_get_time",
           "paraiso_wave_workspace_bytes", "paraiso_wave_prepare", "paraiso_wave_run",
           "paraiso_wave_advance", "paraiso_mlp_sizes", "paraiso_mlp_forward", "paraiso_mlp_loss_grad",
           "paraiso_mlp_adam", "paraiso_cfl_dt_static")


class ParaisoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"paraiso status {code}: {msg}")
        self.code = code


class NonFiniteError(ParaisoError, FloatingPointError):
    pass


class paraiso_mesh(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("dx", ctypes.c_double * 3), ("gamma", ctypes.c_double), ("bc", ctypes.c_int32 * 3),
                ("order", ctypes.c_int32), ("state", (ctypes.c_void_p * 5) * 2)]


class paraiso_analytic(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("angle", ctypes.c_double),
                ("amplitude", ctypes.c_double)]

    @classmethod
    def make(cls, kind, angle=0.0, amplitude=0.0):
        a = cls()
        a.kind, a.reserved, a.angle, a.amplitude = int(kind), 0, float(angle), float(amplitude)
        return a


WAVE_MAX_CELLS = 4096


class paraiso_wave(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("c", ctypes.c_double), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("f", ctypes.c_void_p), ("g", ctypes.c_void_p), ("energy", ctypes.c_void_p)]


class paraiso_variant(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32 * 3), ("lds", ctypes.c_int32), ("fuse", ctypes.c_int32),
                ("waves_per_eu", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("manifest", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"tile": tuple(self.tile), "lds": self.lds, "fuse": self.fuse,
                "waves_per_eu": self.waves_per_eu, "threads": self.threads,
                "persistent": self.persistent, "manifest": self.manifest}

    @classmethod
    def make(cls, tile=(32, 16, 1), lds=1, fuse=1, waves_per_eu=0, threads=0, persistent=0, manifest=0):
        v = cls()
        t = tuple(tile) + (1,) * (3 - len(tile))
        for a in range(3):
            v.tile[a] = int(t[a])
        v.lds, v.fuse, v.waves_per_eu = int(lds), int(fuse), int(waves_per_eu)
        v.threads, v.persistent, v.manifest = int(threads), int(persistent), int(manifest)
        return v


_lib = None


def load(path: str | None = None):
    """Load libparaiso.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with `python -m paper_1204_4779_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl, szt = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    mp = ctypes.POINTER(paraiso_mesh)
    varp = ctypes.POINTER(paraiso_variant)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "paraiso_workspace_bytes": ([mp, i32, ctypes.POINTER(szt)], i32),
        "paraiso_init": ([mp, i32, vp, szt, vp, ctypes.POINTER(vp)], i32),
        "paraiso_set_variant": ([vp, varp], i32),
        "paraiso_get_variant": ([vp, varp], i32),
        "paraiso_default_variant": ([mp, i32, varp], i32),
        "paraiso_cfl_dt": ([vp, dbl, dp], i32),
        "paraiso_cfl_dt_static": ([ctypes.POINTER(paraiso_mesh), i32, i32, dbl, dp, vp], i32),
        "paraiso_step": ([vp, dp], i32),
        "paraiso_advance": ([vp, dbl, dbl, i64, dp, ctypes.POINTER(i64)], i32),
        "paraiso_current": ([vp, ctypes.POINTER(i32)], i32),
        "paraiso_totals": ([vp, dp], i32),
        "paraiso_set_analytic": ([vp, i32, ctypes.POINTER(paraiso_analytic)], i32),
        "paraiso_exact_state": ([vp, i32, dbl, i32], i32),
        "paraiso_set_time": ([vp, dp], i32),
        "paraiso_wave_workspace_bytes": ([i32, ctypes.POINTER(szt)], i32),
        "paraiso_wave_prepare": ([ctypes.POINTER(paraiso_wave), i32, vp, szt, vp], i32),
        "paraiso_wave_run": ([vp, i32, i64, i64, vp], i32),
        "paraiso_wave_advance": ([ctypes.POINTER(paraiso_wave), i32, i64, vp, szt, vp], i32),
        "paraiso_get_time": ([vp, dp], i32),
        "paraiso_destroy": ([vp], i32),
        "paraiso_last_error": ([], ctypes.c_char_p),
        "paraiso_version": ([], ctypes.c_char_p),
        "paraiso_mlp_sizes": ([i32, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(szt)], i32),
        "paraiso_mlp_forward": ([vp, i32, i32, i32, vp, vp, vp, szt, vp], i32),
        "paraiso_mlp_loss_grad": ([vp, vp, i32, i32, i32, vp, vp, vp, vp, szt, vp], i32),
        "paraiso_mlp_adam": ([vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, i32, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        msg = load().paraiso_last_error().decode()
        if rc == ERR_NONFINITE:
            raise NonFiniteError(rc, msg)
        raise ParaisoError(rc, msg)


def _dbl_array(values):
    arr = (ctypes.c_double * len(values))(*[float(v) for v in values])
    return arr


# --- the C entry points, one Python function each ----------------------------------------

def paraiso_workspace_bytes(meshes) -> int:
    arr = (paraiso_mesh * len(meshes))(*meshes)
    out = ctypes.c_size_t()
    _check(load().paraiso_workspace_bytes(arr, len(meshes), ctypes.byref(out)))
    return out.value


def paraiso_default_variant(meshes) -> paraiso_variant:
    arr = (paraiso_mesh * len(meshes))(*meshes)
    v = paraiso_variant()
    _check(load().paraiso_default_variant(arr, len(meshes), ctypes.byref(v)))
    return v


def paraiso_init(meshes, workspace_ptr: int, workspace_bytes: int, stream_ptr: int) -> int:
    arr = (paraiso_mesh * len(meshes))(*meshes)
    ctx = ctypes.c_void_p()
    _check(load().paraiso_init(arr, len(meshes), ctypes.c_void_p(workspace_ptr), workspace_bytes,
                               ctypes.c_void_p(stream_ptr), ctypes.byref(ctx)))
    return ctx.value


def paraiso_set_variant(ctx: int, v: paraiso_variant):
    _check(load().paraiso_set_variant(ctypes.c_void_p(ctx), ctypes.byref(v)))


def paraiso_get_variant(ctx: int) -> paraiso_variant:
    v = paraiso_variant()
    _check(load().paraiso_get_variant(ctypes.c_void_p(ctx), ctypes.byref(v)))
    return v


def paraiso_cfl_dt(ctx: int, cfl: float, count: int = 1) -> list:
    out = (ctypes.c_double * count)()
    _check(load().paraiso_cfl_dt(ctypes.c_void_p(ctx), float(cfl), out))
    return list(out)


def paraiso_cfl_dt_static(meshes, buffer: int, cfl: float, stream: int) -> list:
    """dt per mesh from the state in `buffer` of each descriptor, without a context
    (the library's fixed device scratch; see include/paraiso.h)."""
    arr = (paraiso_mesh * len(meshes))(*meshes)
    out = (ctypes.c_double * len(meshes))()
    _check(load().paraiso_cfl_dt_static(arr, len(meshes), int(buffer), float(cfl), out, ctypes.c_void_p(stream)))
    return list(out)


def paraiso_step(ctx: int, dts) -> None:
    _check(load().paraiso_step(ctypes.c_void_p(ctx), _dbl_array(dts)))


def paraiso_advance(ctx: int, t_end: float, cfl: float, max_steps: int, t0s) -> tuple:
    """(t, steps) per mesh.  A non-physical state raises NonFiniteError whose
    `t` and `steps` hold each mesh's time and step count at return (the
    failing mesh's: those of the step that produced the state)."""
    t = _dbl_array(t0s)
    steps = (ctypes.c_int64 * len(t0s))()
    rc = load().paraiso_advance(ctypes.c_void_p(ctx), float(t_end), float(cfl), int(max_steps), t, steps)
    try:
        _check(rc)
    except NonFiniteError as e:
        e.t, e.steps = list(t), list(steps)
        raise
    return list(t), list(steps)


def paraiso_current(ctx: int) -> int:
    i = ctypes.c_int32()
    _check(load().paraiso_current(ctypes.c_void_p(ctx), ctypes.byref(i)))
    return i.value


def paraiso_totals(ctx: int, count: int, nf: int) -> list:
    out = (ctypes.c_double * (count * nf))()
    _check(load().paraiso_totals(ctypes.c_void_p(ctx), out))
    return [list(out[m * nf:(m + 1) * nf]) for m in range(count)]


def paraiso_set_analytic(ctx: int, mesh: int, an: paraiso_analytic) -> None:
    _check(load().paraiso_set_analytic(ctypes.c_void_p(ctx), int(mesh), ctypes.byref(an)))


def paraiso_exact_state(ctx: int, mesh: int, t: float, buffer: int) -> None:
    _check(load().paraiso_exact_state(ctypes.c_void_p(ctx), int(mesh), float(t), int(buffer)))


def paraiso_set_time(ctx: int, ts) -> None:
    _check(load().paraiso_set_time(ctypes.c_void_p(ctx), _dbl_array(ts)))


def paraiso_get_time(ctx: int, count: int = 1) -> list:
    out = (ctypes.c_double * count)()
    _check(load().paraiso_get_time(ctypes.c_void_p(ctx), out))
    return list(out)


def paraiso_wave_workspace_bytes(count: int) -> int:
    out = ctypes.c_size_t()
    _check(load().paraiso_wave_workspace_bytes(int(count), ctypes.byref(out)))
    return out.value


def paraiso_wave_prepare(lines, workspace_ptr: int, workspace_bytes: int, stream_ptr: int) -> None:
    arr = (paraiso_wave * len(lines))(*lines)
    _check(load().paraiso_wave_prepare(arr, len(lines), ctypes.c_void_p(workspace_ptr), int(workspace_bytes),
                                       ctypes.c_void_p(stream_ptr)))


def paraiso_wave_run(workspace_ptr: int, count: int, steps: int, max_cells: int, stream_ptr: int) -> None:
    _check(load().paraiso_wave_run(ctypes.c_void_p(workspace_ptr), int(count), int(steps), int(max_cells),
                                   ctypes.c_void_p(stream_ptr)))


def paraiso_wave_advance(lines, steps: int, workspace_ptr: int, workspace_bytes: int, stream_ptr: int) -> None:
    arr = (paraiso_wave * len(lines))(*lines)
    _check(load().paraiso_wave_advance(arr, len(lines), int(steps), ctypes.c_void_p(workspace_ptr),
                                       int(workspace_bytes), ctypes.c_void_p(stream_ptr)))


def paraiso_destroy(ctx: int) -> None:
    _check(load().paraiso_destroy(ctypes.c_void_p(ctx)))


def paraiso_version() -> str:
    return load().paraiso_version().decode()


def paraiso_mlp_sizes(in_dim: int, hidden: int, batch: int) -> tuple:
    n = ctypes.c_int64()
    ws = ctypes.c_size_t()
    _check(load().paraiso_mlp_sizes(in_dim, hidden, batch, ctypes.byref(n), ctypes.byref(ws)))
    return n.value, ws.value


def paraiso_mlp_forward(X_ptr, batch, in_dim, hidden, params_ptr, y_ptr, ws_ptr, ws_bytes, stream_ptr):
    _check(load().paraiso_mlp_forward(X_ptr, batch, in_dim, hidden, params_ptr, y_ptr, ws_ptr, ws_bytes,
                                      stream_ptr))


def paraiso_mlp_loss_grad(X_ptr, T_ptr, batch, in_dim, hidden, params_ptr, grad_ptr, loss_ptr, ws_ptr, ws_bytes,
                          stream_ptr):
    _check(load().paraiso_mlp_loss_grad(X_ptr, T_ptr, batch, in_dim, hidden, params_ptr, grad_ptr, loss_ptr,
                                        ws_ptr, ws_bytes, stream_ptr))


def paraiso_mlp_adam(p_ptr, g_ptr, m_ptr, v_ptr, n, lr, beta1, beta2, eps, step, stream_ptr):
    _check(load().paraiso_mlp_adam(p_ptr, g_ptr, m_ptr, v_ptr, n, lr, beta1, beta2, eps, step, stream_ptr))


# --- torch-side convenience ----------------------------------------------------------------

@dataclass
class MeshSpec:
    ndim: int
    n: tuple              # (nx, ny, nz), 1 for unused axes
    gamma: float
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    dx: tuple | None = None
    order: int = 2        # reconstruction: 2 minbee piecewise linear, 1 piecewise constant

    def n3(self):
        return tuple(int(v) for v in self.n) + (1,) * (3 - len(self.n))

    def dx3(self):
        n = self.n3()
        if self.dx is None:
            return tuple(1.0 / n[a] if a < self.ndim else 1.0 for a in range(3))
        return tuple(float(v) for v in self.dx) + (1.0,) * (3 - len(self.dx))


class Solver:
    """One context over one mesh or a batch; state buffers are torch tensors of shape
    (d+2, nz, ny, nx) (leading axes dropped for d < 3), two per mesh."""

    def __init__(self, specs, dtype: str = "f32", device=None, stream=None, workspace_fill: int | None = None):
        import torch
        self.torch = torch
        if isinstance(specs, MeshSpec):
            specs = [specs]
        self.specs = list(specs)
        self.dtype = dtype
        tdt = torch.float32 if dtype == "f32" else torch.float64
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.ndim = self.specs[0].ndim
        self.nf = self.ndim + 2
        self.buffers = []
        meshes = []
        for sp in self.specs:
            n = sp.n3()
            dims = tuple(reversed(n[: sp.ndim]))
            cells = n[0] * n[1] * n[2]
            padded = (cells + 63) // 64 * 64      # every field starts 256-byte aligned
            inner = [1]                           # contiguous strides of one field, x fastest
            for extent in reversed(dims[1:]):
                inner.insert(0, inner[0] * extent)
            strides = (padded,) + tuple(inner)
            pair = []
            for _ in range(2):
                store = torch.zeros((self.nf, padded), dtype=tdt, device=dev)
                pair.append(torch.as_strided(store, (self.nf,) + dims, strides))
            b0, b1 = pair
            self.buffers.append((b0, b1))
            m = paraiso_mesh()
            m.ndim = sp.ndim
            m.dtype = F32 if dtype == "f32" else F64
            dx = sp.dx3()
            bc = tuple(sp.bc) + (PERIODIC,) * (3 - len(sp.bc))
            for a in range(3):
                m.n[a] = n[a]
                m.dx[a] = dx[a]
                m.bc[a] = bc[a]
            m.gamma = float(sp.gamma)
            m.order = int(sp.order)
            for b, buf in enumerate((b0, b1)):
                for q in range(self.nf):
                    m.state[b][q] = buf[q].data_ptr()   # field q: contiguous, 256-byte aligned
            meshes.append(m)
        self.meshes = meshes
        self.ws_bytes = paraiso_workspace_bytes(meshes)
        if workspace_fill is None:
            self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        else:   # a byte pattern in the whole workspace (tests: reads of unwritten workspace show)
            self.workspace = torch.full((self.ws_bytes + 256,), int(workspace_fill), dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        self.ctx = paraiso_init(meshes, self.ws_ptr, self.ws_bytes, stream.cuda_stream)

    @property
    def count(self) -> int:
        return len(self.specs)

    def close(self):
        if getattr(self, "ctx", None):
            paraiso_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_variant(self, v: paraiso_variant | dict):
        if isinstance(v, dict):
            v = paraiso_variant.make(**v)
        paraiso_set_variant(self.ctx, v)

    def variant(self) -> dict:
        return paraiso_get_variant(self.ctx).as_dict()

    def current(self) -> int:
        return paraiso_current(self.ctx)

    def upload(self, states):
        """Copy initial states (array-likes of shape (d+2, ...)) into the current buffer."""
        torch = self.torch
        if self.count == 1 and not isinstance(states, (list, tuple)):
            states = [states]
        cur = self.current()
        for (bufs, st) in zip(self.buffers, states):
            t = torch.as_tensor(st).to(dtype=bufs[0].dtype)
            bufs[cur].copy_(t.reshape(bufs[cur].shape))
        torch.cuda.synchronize(self.device)

    def state(self, m: int = 0):
        return self.buffers[m][self.current()]

    def cfl_dt(self, cfl: float) -> list:
        return paraiso_cfl_dt(self.ctx, cfl, self.count)

    def step(self, dts):
        if not isinstance(dts, (list, tuple)):
            dts = [dts] * self.count
        paraiso_step(self.ctx, dts)

    def advance(self, t_end: float, cfl: float, max_steps: int = (1 << 62), t0=None):
        t0 = [0.0] * self.count if t0 is None else list(t0)
        return paraiso_advance(self.ctx, t_end, cfl, max_steps, t0)

    def totals(self) -> list:
        return paraiso_totals(self.ctx, self.count, self.nf)

    def set_analytic(self, kind: int, angle: float = 0.0, amplitude: float = 0.0, mesh: int = 0):
        paraiso_set_analytic(self.ctx, mesh, paraiso_analytic.make(kind, angle, amplitude))

    def fill_exact(self, t: float, mesh: int = 0, buffer: int | None = None):
        """Exact state of the mesh's problem at time t into the current buffer (or `buffer`)."""
        paraiso_exact_state(self.ctx, mesh, t, self.current() if buffer is None else buffer)

    def set_time(self, ts):
        if not isinstance(ts, (list, tuple)):
            ts = [ts] * self.count
        paraiso_set_time(self.ctx, ts)

    def time(self) -> list:
        return paraiso_get_time(self.ctx, self.count)


class WaveLines:
    """A batch of periodic lines for paraiso_wave_advance: f, g and the energy
    history as FP64 torch tensors on the current device, torch's current stream."""

    def __init__(self, fs, gs, c, dx, dt, steps_capacity: int, device=None):
        import torch
        self.torch = torch
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        count = len(fs)
        per = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * count
        self.c, self.dx, self.dt = per(c), per(dx), per(dt)
        self.f = [torch.as_tensor(v, dtype=torch.float64).to(dev).contiguous() for v in fs]
        self.g = [torch.as_tensor(v, dtype=torch.float64).to(dev).contiguous() for v in gs]
        self.energy = [torch.zeros(max(int(steps_capacity), 1), dtype=torch.float64, device=dev)
                       for _ in range(count)]
        self.capacity = int(steps_capacity)
        self.ws_bytes = paraiso_wave_workspace_bytes(count)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        self.ws_ptr = (self.workspace.data_ptr() + 255) & ~255
        self.recording = None   # set by prepare()

    def prepare(self, record_energy: bool = True):
        """Upload the line table; run() then enqueues steps without host work."""
        paraiso_wave_prepare(self._lines(record_energy), self.ws_ptr, self.ws_bytes,
                             self.torch.cuda.current_stream(self.device).cuda_stream)
        self.recording = record_energy

    def run(self, steps: int):
        if self.recording is None:
            raise RuntimeError("WaveLines.run: call prepare() first (it uploads the line table)")
        if self.recording and steps > self.capacity:
            raise ValueError("more steps than the energy buffers hold")
        paraiso_wave_run(self.ws_ptr, len(self.f), steps, max(x.numel() for x in self.f),
                         self.torch.cuda.current_stream(self.device).cuda_stream)

    def _lines(self, record_energy: bool):
        lines = []
        for k in range(len(self.f)):
            w = paraiso_wave()
            w.n, w.c, w.dx, w.dt = self.f[k].numel(), self.c[k], self.dx[k], self.dt[k]
            w.f, w.g = self.f[k].data_ptr(), self.g[k].data_ptr()
            w.energy = self.energy[k].data_ptr() if record_energy else None
            lines.append(w)
        return lines

    def advance(self, steps: int, record_energy: bool = True):
        if record_energy and steps > self.capacity:
            raise ValueError("more steps than the energy buffers hold")
        stream = self.torch.cuda.current_stream(self.device)
        paraiso_wave_advance(self._lines(record_energy), steps, self.ws_ptr, self.ws_bytes, stream.cuda_stream)

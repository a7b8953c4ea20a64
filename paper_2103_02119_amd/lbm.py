"""Python binding of the C ABI in include/lbm.h (liblbm.so).

Argument marshalling only: every function here forwards to the HIP library
with the same name and turns a negative status into LbmError.  There is no
CPU fallback -- if liblbm.so is missing or no GPU is usable, calls raise.
PyTorch is used (optionally) only to own the device population buffers and
to supply the HIP stream the library enqueues on.

Host arrays are numpy float64, C order: scalar fields (ny, nx), populations
(9, ny, nx).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_UNSTABLE, LBM_E_STATE = 0, -1, -2, -3, -4, -5
LBM_BC_PERIODIC, LBM_BC_WALL, LBM_BC_MOVING_WALL = 0, 1, 2
LBM_FACE_XMIN, LBM_FACE_XMAX, LBM_FACE_YMIN, LBM_FACE_YMAX = 0, 1, 2, 3
LBM_RC, LBM_RNR = 0, 1
LBM_FP64, LBM_FP32_DEV, LBM_FP64_DEV, LBM_FP32_DEV_F64 = 0, 1, 2, 3
LBM_FORM_AUTO, LBM_FORM_REGISTER, LBM_FORM_STAGED = 0, 1, 2

EXPORTS = ("lbm_default_opts", "lbm_required_bytes", "lbm_create", "lbm_set_fields", "lbm_step",
           "lbm_set_steps_per_launch", "lbm_steps_per_launch", "lbm_set_two_step_form",
           "lbm_two_step_form",
           "lbm_moments", "lbm_stress", "lbm_residual", "lbm_sums", "lbm_check_async",
           "lbm_check_result", "lbm_check_into", "lbm_get_populations", "lbm_set_populations",
           "lbm_set_mask", "lbm_set_rates", "lbm_set_force", "lbm_step_forced", "lbm_smooth_step",
           "lbm_stream_copy", "lbm_steps_done", "lbm_launch_shape", "lbm_last_error",
           "lbm_destroy")
BATCH_EXPORTS = ("lbm_batch_default_opts", "lbm_batch_create", "lbm_batch_set_fields",
                 "lbm_batch_set_mask", "lbm_batch_set_rates", "lbm_batch_smooth_step",
                 "lbm_batch_set_active", "lbm_batch_step", "lbm_batch_residuals",
                 "lbm_batch_run_to_steady", "lbm_batch_moments", "lbm_batch_get_populations",
                 "lbm_batch_set_populations", "lbm_batch_steps_done", "lbm_batch_autotune",
                 "lbm_batch_uses_tile_kernel", "lbm_batch_steps_per_launch",
                 "lbm_batch_two_step_form",
                 "lbm_batch_launch_shape", "lbm_batch_last_error", "lbm_batch_destroy")


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class lbm_bc(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int * 4), ("u_wall", (ctypes.c_double * 2) * 4)]


class lbm_opts(ctypes.Structure):
    _fields_ = [
        ("cs2", ctypes.c_double),
        ("force", ctypes.c_double * 2),
        ("rho0", ctypes.c_double),
        ("collision", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("corrections", ctypes.c_int),
        ("rows_per_wave", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("f_a", ctypes.c_void_p),
        ("f_b", ctypes.c_void_p),
        ("f_bytes", ctypes.c_size_t),
    ]


class lbm_case(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("r", ctypes.c_double),
        ("rates", ctypes.c_double * 9),
        ("bc", lbm_bc),
        ("cs2", ctypes.c_double),
        ("force", ctypes.c_double * 2),
        ("rho0", ctypes.c_double),
    ]


class lbm_batch_opts(ctypes.Structure):
    _fields_ = [
        ("collision", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("corrections", ctypes.c_int),
        ("rows_per_wave", ctypes.c_int),
        ("workgroups", ctypes.c_int),
        ("graph_steps", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("tile_kernel", ctypes.c_int),
        ("steps_per_launch", ctypes.c_int),
        ("two_step_form", ctypes.c_int),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_CTX = ctypes.c_void_p


def load():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it first "
                           "(python -m paper_2103_02119_amd.build)")
    # PyTorch-ROCm ships its own HIP and HSA runtimes.  Load them first, so
    # that the library binds to the runtime already in the process: if the
    # system runtime came first, torch's own would later fail to open the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    L.lbm_default_opts.argtypes = [ctypes.POINTER(lbm_opts)]
    L.lbm_default_opts.restype = None
    L.lbm_required_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_size_t)]
    L.lbm_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _D,
                             ctypes.POINTER(lbm_bc), ctypes.POINTER(lbm_opts),
                             ctypes.POINTER(_CTX)]
    L.lbm_set_fields.argtypes = [_CTX, _D, _D, _D]
    L.lbm_step.argtypes = [_CTX, ctypes.c_long]
    L.lbm_set_steps_per_launch.argtypes = [_CTX, ctypes.c_int]
    L.lbm_set_steps_per_launch.restype = ctypes.c_int
    L.lbm_steps_per_launch.argtypes = [_CTX]
    L.lbm_steps_per_launch.restype = ctypes.c_int
    L.lbm_set_two_step_form.argtypes = [_CTX, ctypes.c_int]
    L.lbm_set_two_step_form.restype = ctypes.c_int
    L.lbm_two_step_form.argtypes = [_CTX]
    L.lbm_two_step_form.restype = ctypes.c_int
    L.lbm_check_into.argtypes = [_CTX, ctypes.c_void_p]
    L.lbm_check_into.restype = ctypes.c_int
    L.lbm_stream_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                  ctypes.c_void_p]
    L.lbm_stream_copy.restype = ctypes.c_int
    L.lbm_moments.argtypes = [_CTX, _D, _D, _D]
    L.lbm_stress.argtypes = [_CTX, _D, _D, _D]
    L.lbm_residual.argtypes = [_CTX, _D]
    L.lbm_sums.argtypes = [_CTX, _D]
    L.lbm_check_async.argtypes = [_CTX]
    L.lbm_check_async.restype = ctypes.c_int
    L.lbm_check_result.argtypes = [_CTX, ctypes.POINTER(ctypes.c_double), _D,
                                   ctypes.POINTER(ctypes.c_long)]
    L.lbm_check_result.restype = ctypes.c_int
    L.lbm_get_populations.argtypes = [_CTX, _D]
    L.lbm_set_populations.argtypes = [_CTX, _D]
    _U8 = ctypes.POINTER(ctypes.c_ubyte)
    L.lbm_set_mask.argtypes = [_CTX, _U8]
    L.lbm_set_mask.restype = ctypes.c_int
    L.lbm_set_rates.argtypes = [_CTX, _D]
    L.lbm_set_rates.restype = ctypes.c_int
    L.lbm_set_force.argtypes = [_CTX, ctypes.c_double, ctypes.c_double]
    L.lbm_set_force.restype = ctypes.c_int
    L.lbm_step_forced.argtypes = [_CTX, ctypes.c_long, _D, _D]
    L.lbm_step_forced.restype = ctypes.c_int
    L.lbm_smooth_step.argtypes = [_CTX]
    L.lbm_smooth_step.restype = ctypes.c_int
    L.lbm_steps_done.argtypes = [_CTX]
    L.lbm_steps_done.restype = ctypes.c_long
    L.lbm_launch_shape.argtypes = [_CTX, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int)]
    L.lbm_last_error.argtypes = [_CTX]
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_destroy.argtypes = [_CTX]
    for name in ("lbm_required_bytes", "lbm_create", "lbm_set_fields", "lbm_step", "lbm_moments",
                 "lbm_stress", "lbm_residual", "lbm_sums", "lbm_get_populations", "lbm_set_populations",
                 "lbm_launch_shape", "lbm_destroy"):
        getattr(L, name).restype = ctypes.c_int
    _I = ctypes.POINTER(ctypes.c_int)
    _B = ctypes.c_void_p
    L.lbm_batch_default_opts.argtypes = [ctypes.POINTER(lbm_batch_opts)]
    L.lbm_batch_default_opts.restype = None
    L.lbm_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(lbm_case),
                                   ctypes.POINTER(lbm_batch_opts), ctypes.POINTER(_B)]
    L.lbm_batch_set_fields.argtypes = [_B, ctypes.c_int, _D, _D, _D]
    L.lbm_batch_set_mask.argtypes = [_B, ctypes.c_int, _U8]
    L.lbm_batch_set_mask.restype = ctypes.c_int
    L.lbm_batch_set_rates.argtypes = [_B, ctypes.c_int, _D]
    L.lbm_batch_set_rates.restype = ctypes.c_int
    L.lbm_batch_smooth_step.argtypes = [_B]
    L.lbm_batch_smooth_step.restype = ctypes.c_int
    L.lbm_batch_set_active.argtypes = [_B, _I]
    L.lbm_batch_step.argtypes = [_B, ctypes.c_long]
    L.lbm_batch_residuals.argtypes = [_B, _D]
    L.lbm_batch_run_to_steady.argtypes = [_B, ctypes.c_double, ctypes.c_long, ctypes.c_long,
                                          ctypes.POINTER(ctypes.c_long)]
    L.lbm_batch_moments.argtypes = [_B, ctypes.c_int, _D, _D, _D]
    L.lbm_batch_get_populations.argtypes = [_B, ctypes.c_int, _D]
    L.lbm_batch_set_populations.argtypes = [_B, ctypes.c_int, _D]
    L.lbm_batch_steps_done.argtypes = [_B, ctypes.c_int]
    L.lbm_batch_steps_done.restype = ctypes.c_long
    L.lbm_batch_autotune.argtypes = [_B, ctypes.c_int, _I, _I]
    L.lbm_batch_launch_shape.argtypes = [_B, _I, _I, _I]
    L.lbm_batch_uses_tile_kernel.argtypes = [_B]
    L.lbm_batch_uses_tile_kernel.restype = ctypes.c_int
    L.lbm_batch_steps_per_launch.argtypes = [_B]
    L.lbm_batch_steps_per_launch.restype = ctypes.c_int
    L.lbm_batch_two_step_form.argtypes = [_B]
    L.lbm_batch_two_step_form.restype = ctypes.c_int
    L.lbm_batch_last_error.argtypes = [_B]
    L.lbm_batch_last_error.restype = ctypes.c_char_p
    L.lbm_batch_destroy.argtypes = [_B]
    for name in ("lbm_batch_create", "lbm_batch_set_fields", "lbm_batch_set_active",
                 "lbm_batch_step", "lbm_batch_residuals", "lbm_batch_run_to_steady",
                 "lbm_batch_moments", "lbm_batch_get_populations", "lbm_batch_set_populations",
                 "lbm_batch_autotune", "lbm_batch_launch_shape", "lbm_batch_destroy"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc, ctx=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error(ctx).decode(errors="replace")
        raise LbmError(rc, msg)


def _in(arr, shape):
    if arr is None:
        return None, None
    a = np.ascontiguousarray(arr, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a, a.ctypes.data_as(_D)


# ----------------------------------------------------------- same-name calls

def lbm_default_opts() -> lbm_opts:
    o = lbm_opts()
    load().lbm_default_opts(ctypes.byref(o))
    return o


def lbm_required_bytes(nx: int, ny: int, precision: int) -> int:
    n = ctypes.c_size_t()
    _check(load().lbm_required_bytes(nx, ny, precision, ctypes.byref(n)))
    return n.value


def make_bc(types=(LBM_BC_PERIODIC,) * 4, u_wall=((0.0, 0.0),) * 4) -> lbm_bc:
    b = lbm_bc()
    for f in range(4):
        b.type[f] = int(types[f])
        b.u_wall[f][0] = float(u_wall[f][0])
        b.u_wall[f][1] = float(u_wall[f][1])
    return b


def lbm_create(nx: int, ny: int, r: float, rates, bc: lbm_bc, opts: lbm_opts | None = None):
    rates_arr = (ctypes.c_double * 9)(*[float(w) for w in rates])
    ctx = _CTX()
    rc = load().lbm_create(int(nx), int(ny), float(r), rates_arr, ctypes.byref(bc),
                           ctypes.byref(opts) if opts is not None else None, ctypes.byref(ctx))
    _check(rc, None)
    return ctx


def lbm_set_fields(ctx, nx, ny, rho=None, ux=None, uy=None):
    keep = [_in(v, (ny, nx)) for v in (rho, ux, uy)]
    _check(load().lbm_set_fields(ctx, *[k[1] for k in keep]), ctx)


def lbm_step(ctx, n: int):
    _check(load().lbm_step(ctx, int(n)), ctx)


def lbm_set_steps_per_launch(ctx, k: int):
    _check(load().lbm_set_steps_per_launch(ctx, int(k)), ctx)


def lbm_steps_per_launch(ctx) -> int:
    k = load().lbm_steps_per_launch(ctx)
    if k < 0:
        raise LbmError(k, "NULL context")
    return k


def lbm_set_two_step_form(ctx, form: int):
    _check(load().lbm_set_two_step_form(ctx, int(form)), ctx)


def lbm_two_step_form(ctx) -> int:
    f = load().lbm_two_step_form(ctx)
    if f < 0:
        raise LbmError(f, "NULL context")
    return f


def lbm_moments(ctx, nx, ny):
    rho, ux, uy = (np.empty((ny, nx)) for _ in range(3))
    _check(load().lbm_moments(ctx, rho.ctypes.data_as(_D), ux.ctypes.data_as(_D),
                              uy.ctypes.data_as(_D)), ctx)
    return rho, ux, uy


def lbm_stress(ctx, nx, ny):
    """(sxx, syy, sxy), each (ny, nx), of the current time level."""
    out = tuple(np.empty((ny, nx)) for _ in range(3))
    _check(load().lbm_stress(ctx, *(o.ctypes.data_as(_D) for o in out)), ctx)
    return out


def lbm_residual(ctx) -> float:
    R = ctypes.c_double()
    _check(load().lbm_residual(ctx, ctypes.byref(R)), ctx)
    return R.value


def lbm_sums(ctx):
    out = np.zeros(3)
    _check(load().lbm_sums(ctx, out.ctypes.data_as(_D)), ctx)
    return out


def lbm_check_async(ctx):
    _check(load().lbm_check_async(ctx), ctx)


def lbm_check_result(ctx):
    """(R, sums, step) of the latest lbm_check_async."""
    R, step, out = ctypes.c_double(), ctypes.c_long(), np.zeros(3)
    _check(load().lbm_check_result(ctx, ctypes.byref(R), out.ctypes.data_as(_D),
                                   ctypes.byref(step)), ctx)
    return R.value, out, step.value


def lbm_check_into(ctx, out_ptr: int):
    """Enqueue the fused check with its results written to device memory at
    out_ptr (8 doubles, e.g. a torch float64 tensor's data_ptr())."""
    _check(load().lbm_check_into(ctx, ctypes.c_void_p(int(out_ptr))), ctx)


def lbm_stream_copy(dst_ptr: int, src_ptr: int, nbytes: int, workgroups: int = 0, stream=None):
    """The library's streaming copy kernel between two device buffers."""
    _check(load().lbm_stream_copy(ctypes.c_void_p(int(dst_ptr)), ctypes.c_void_p(int(src_ptr)),
                                  int(nbytes), int(workgroups),
                                  None if stream is None else ctypes.c_void_p(int(stream))), None)


def lbm_get_populations(ctx, nx, ny):
    f = np.empty((9, ny, nx))
    _check(load().lbm_get_populations(ctx, f.ctypes.data_as(_D)), ctx)
    return f


def lbm_set_populations(ctx, nx, ny, f):
    a, p = _in(f, (9, ny, nx))
    _check(load().lbm_set_populations(ctx, p), ctx)


def _mask(mask, shape):
    if mask is None:
        return None, None
    m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
    if m.shape != shape:
        raise ValueError(f"expected mask shape {shape}, got {m.shape}")
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


def lbm_set_mask(ctx, nx, ny, mask=None):
    keep, p = _mask(mask, (ny, nx))
    _check(load().lbm_set_mask(ctx, p), ctx)


def lbm_set_force(ctx, fx, fy=0.0):
    _check(load().lbm_set_force(ctx, float(fx), float(fy)), ctx)


def lbm_step_forced(ctx, fx, fy=None):
    ax = np.ascontiguousarray(fx, dtype=np.float64)
    ay = None if fy is None else np.ascontiguousarray(fy, dtype=np.float64)
    if ay is not None and ay.shape != ax.shape:
        raise ValueError("fx and fy must have the same length")
    _check(load().lbm_step_forced(ctx, ax.size, ax.ctypes.data_as(_D),
                                  None if ay is None else ay.ctypes.data_as(_D)), ctx)


def lbm_smooth_step(ctx):
    _check(load().lbm_smooth_step(ctx), ctx)


def lbm_set_rates(ctx, rates):
    arr = (ctypes.c_double * 9)(*[float(w) for w in rates])
    _check(load().lbm_set_rates(ctx, arr), ctx)


def lbm_steps_done(ctx) -> int:
    return load().lbm_steps_done(ctx)


def lbm_launch_shape(ctx):
    r, w = ctypes.c_int(), ctypes.c_int()
    _check(load().lbm_launch_shape(ctx, ctypes.byref(r), ctypes.byref(w)), ctx)
    return r.value, w.value


def lbm_last_error(ctx=None) -> str:
    return load().lbm_last_error(ctx).decode(errors="replace")


def lbm_destroy(ctx):
    if ctx:
        load().lbm_destroy(ctx)


# ----------------------------------------------------------- convenience

class Lattice:
    """Owns one lbm_ctx.  With torch_buffers=True the two population buffers
    are torch CUDA tensors and the library runs on torch's current stream."""

    def __init__(self, nx, ny, r, rates, bc_types=(LBM_BC_PERIODIC,) * 4,
                 u_wall=((0.0, 0.0),) * 4, cs2=0.0, force=(0.0, 0.0), rho0=1.0,
                 collision=LBM_RC, precision=LBM_FP64, corrections=True, rows_per_wave=0,
                 torch_buffers=True):
        self.nx, self.ny, self.r = int(nx), int(ny), float(r)
        o = lbm_default_opts()
        o.cs2 = float(cs2)
        o.force[0], o.force[1] = float(force[0]), float(force[1])
        o.rho0 = float(rho0)
        o.collision = int(collision)
        o.precision = int(precision)
        o.corrections = 1 if corrections else 0
        o.rows_per_wave = int(rows_per_wave)
        self._buffers = None
        if torch_buffers:
            import torch
            nbytes = lbm_required_bytes(self.nx, self.ny, int(precision))
            self._buffers = [torch.empty(nbytes, dtype=torch.uint8, device="cuda")
                             for _ in range(2)]
            o.f_a = self._buffers[0].data_ptr()
            o.f_b = self._buffers[1].data_ptr()
            o.f_bytes = nbytes
            o.stream = torch.cuda.current_stream().cuda_stream
        self.opts = o
        self.ctx = lbm_create(self.nx, self.ny, self.r, rates, make_bc(bc_types, u_wall), o)

    def set_fields(self, rho=None, ux=None, uy=None):
        lbm_set_fields(self.ctx, self.nx, self.ny, rho, ux, uy)

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def set_steps_per_launch(self, k):
        lbm_set_steps_per_launch(self.ctx, k)

    def steps_per_launch(self):
        return lbm_steps_per_launch(self.ctx)

    def set_two_step_form(self, form):
        lbm_set_two_step_form(self.ctx, form)

    def two_step_form(self):
        return lbm_two_step_form(self.ctx)

    def check_into(self, out_ptr):
        lbm_check_into(self.ctx, out_ptr)

    def moments(self):
        return lbm_moments(self.ctx, self.nx, self.ny)

    def stress(self):
        return lbm_stress(self.ctx, self.nx, self.ny)

    def residual(self):
        return lbm_residual(self.ctx)

    def sums(self):
        return lbm_sums(self.ctx)

    def check_async(self):
        lbm_check_async(self.ctx)

    def check_result(self):
        return lbm_check_result(self.ctx)

    def get_populations(self):
        return lbm_get_populations(self.ctx, self.nx, self.ny)

    def set_populations(self, f):
        lbm_set_populations(self.ctx, self.nx, self.ny, f)

    def launch_shape(self):
        return lbm_launch_shape(self.ctx)

    def set_mask(self, mask=None):
        lbm_set_mask(self.ctx, self.nx, self.ny, mask)

    def set_rates(self, rates):
        lbm_set_rates(self.ctx, rates)

    def smooth_step(self):
        lbm_smooth_step(self.ctx)

    def set_force(self, fx, fy=0.0):
        lbm_set_force(self.ctx, fx, fy)

    def step_forced(self, fx, fy=None):
        lbm_step_forced(self.ctx, fx, fy)

    @property
    def steps_done(self):
        return lbm_steps_done(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ----------------------------------------------------------- batches (lbm_batch.h)

def _bcheck(rc, b=None):
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_batch_last_error(b).decode(errors="replace"))


def make_case(nx, ny, r, rates, bc_types=(LBM_BC_PERIODIC,) * 4, u_wall=((0.0, 0.0),) * 4,
              cs2=0.0, force=(0.0, 0.0), rho0=1.0) -> lbm_case:
    c = lbm_case()
    c.nx, c.ny, c.r = int(nx), int(ny), float(r)
    for j in range(9):
        c.rates[j] = float(rates[j])
    c.bc = make_bc(bc_types, u_wall)
    c.cs2 = float(cs2)
    c.force[0], c.force[1] = float(force[0]), float(force[1])
    c.rho0 = float(rho0)
    return c


def lbm_batch_default_opts() -> lbm_batch_opts:
    o = lbm_batch_opts()
    load().lbm_batch_default_opts(ctypes.byref(o))
    return o


def lbm_batch_create(cases, opts: lbm_batch_opts | None = None):
    arr = (lbm_case * len(cases))(*cases)
    b = ctypes.c_void_p()
    _bcheck(load().lbm_batch_create(len(cases), arr, ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(b)))
    return b


def lbm_batch_set_fields(b, c, nx, ny, rho=None, ux=None, uy=None):
    keep = [_in(v, (ny, nx)) for v in (rho, ux, uy)]
    _bcheck(load().lbm_batch_set_fields(b, int(c), *[k[1] for k in keep]), b)


def lbm_batch_set_mask(b, c, nx, ny, mask=None):
    keep, p = _mask(mask, (ny, nx))
    _bcheck(load().lbm_batch_set_mask(b, int(c), p), b)


def lbm_batch_smooth_step(b):
    _bcheck(load().lbm_batch_smooth_step(b), b)


def lbm_batch_set_rates(b, c, rates):
    arr = (ctypes.c_double * 9)(*[float(w) for w in rates])
    _bcheck(load().lbm_batch_set_rates(b, int(c), arr), b)


def lbm_batch_set_active(b, active):
    a = (ctypes.c_int * len(active))(*[1 if x else 0 for x in active])
    _bcheck(load().lbm_batch_set_active(b, a), b)


def lbm_batch_step(b, n: int):
    _bcheck(load().lbm_batch_step(b, int(n)), b)


def lbm_batch_residuals(b, ncases):
    R = np.empty(ncases)
    _bcheck(load().lbm_batch_residuals(b, R.ctypes.data_as(_D)), b)
    return R


def lbm_batch_run_to_steady(b, ncases, tol, check_every, max_steps):
    out = (ctypes.c_long * ncases)()
    _bcheck(load().lbm_batch_run_to_steady(b, float(tol), int(check_every), int(max_steps), out), b)
    return np.array(out[:], dtype=np.int64)


def lbm_batch_moments(b, c, nx, ny):
    rho, ux, uy = (np.empty((ny, nx)) for _ in range(3))
    _bcheck(load().lbm_batch_moments(b, int(c), rho.ctypes.data_as(_D), ux.ctypes.data_as(_D),
                                     uy.ctypes.data_as(_D)), b)
    return rho, ux, uy


def lbm_batch_get_populations(b, c, nx, ny):
    f = np.empty((9, ny, nx))
    _bcheck(load().lbm_batch_get_populations(b, int(c), f.ctypes.data_as(_D)), b)
    return f


def lbm_batch_set_populations(b, c, nx, ny, f):
    a, p = _in(f, (9, ny, nx))
    _bcheck(load().lbm_batch_set_populations(b, int(c), p), b)


def lbm_batch_steps_done(b, c) -> int:
    return load().lbm_batch_steps_done(b, int(c))


def lbm_batch_uses_tile_kernel(b) -> bool:
    return load().lbm_batch_uses_tile_kernel(b) == 1


def lbm_batch_steps_per_launch(b) -> int:
    k = load().lbm_batch_steps_per_launch(b)
    if k < 0:
        raise LbmError(k, "NULL batch")
    return k


def lbm_batch_two_step_form(b) -> int:
    f = load().lbm_batch_two_step_form(b)
    if f < 0:
        raise LbmError(f, "NULL batch")
    return f


def lbm_batch_autotune(b, trial_steps=5):
    r, w = ctypes.c_int(), ctypes.c_int()
    _bcheck(load().lbm_batch_autotune(b, int(trial_steps), ctypes.byref(r), ctypes.byref(w)), b)
    return r.value, w.value


def lbm_batch_launch_shape(b):
    r, w, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _bcheck(load().lbm_batch_launch_shape(b, ctypes.byref(r), ctypes.byref(w), ctypes.byref(t)), b)
    return r.value, w.value, t.value


def lbm_batch_last_error(b=None) -> str:
    return load().lbm_batch_last_error(b).decode(errors="replace")


def lbm_batch_destroy(b):
    if b:
        load().lbm_batch_destroy(b)


class Batch:
    """Owns one lbm_batch: cases is a list of lbm_case (see make_case)."""

    def __init__(self, cases, collision=LBM_RC, precision=LBM_FP64, corrections=True,
                 rows_per_wave=0, workgroups=0, graph_steps=0, stream=None, tile_kernel=False,
                 steps_per_launch=0, two_step_form=LBM_FORM_AUTO):
        """stream: a hipStream_t handle (e.g. torch.cuda.Stream().cuda_stream)
        or None for a stream the batch creates; tile_kernel: step with the
        tile kernel from the start (else the autotuner chooses);
        steps_per_launch: 0 automatic (two while no case has a mask), 1, 2;
        two_step_form: LBM_FORM_AUTO, LBM_FORM_REGISTER or LBM_FORM_STAGED."""
        self.shapes = [(c.nx, c.ny) for c in cases]
        self.n = len(cases)
        o = lbm_batch_default_opts()
        o.collision, o.precision = int(collision), int(precision)
        o.corrections = 1 if corrections else 0
        o.rows_per_wave, o.workgroups, o.graph_steps = int(rows_per_wave), int(workgroups), int(graph_steps)
        o.stream = stream
        o.tile_kernel = 1 if tile_kernel else 0
        o.steps_per_launch = int(steps_per_launch)
        o.two_step_form = int(two_step_form)
        self.b = lbm_batch_create(cases, o)

    def set_fields(self, c, rho=None, ux=None, uy=None):
        lbm_batch_set_fields(self.b, c, *self.shapes[c], rho, ux, uy)

    def set_mask(self, c, mask=None):
        lbm_batch_set_mask(self.b, c, *self.shapes[c], mask)

    def set_rates(self, c, rates):
        lbm_batch_set_rates(self.b, c, rates)

    def smooth_step(self):
        lbm_batch_smooth_step(self.b)

    def set_active(self, active):
        lbm_batch_set_active(self.b, active)

    def step(self, n=1):
        lbm_batch_step(self.b, n)

    def residuals(self):
        return lbm_batch_residuals(self.b, self.n)

    def run_to_steady(self, tol, check_every, max_steps):
        return lbm_batch_run_to_steady(self.b, self.n, tol, check_every, max_steps)

    def moments(self, c):
        return lbm_batch_moments(self.b, c, *self.shapes[c])

    def get_populations(self, c):
        return lbm_batch_get_populations(self.b, c, *self.shapes[c])

    def set_populations(self, c, f):
        lbm_batch_set_populations(self.b, c, *self.shapes[c], f)

    def steps_done(self, c):
        return lbm_batch_steps_done(self.b, c)

    def autotune(self, trial_steps=5):
        return lbm_batch_autotune(self.b, trial_steps)

    def uses_tile_kernel(self):
        return lbm_batch_uses_tile_kernel(self.b)

    def steps_per_launch(self):
        return lbm_batch_steps_per_launch(self.b)

    def two_step_form(self):
        return lbm_batch_two_step_form(self.b)

    def launch_shape(self):
        return lbm_batch_launch_shape(self.b)

    def close(self):
        if getattr(self, "b", None):
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

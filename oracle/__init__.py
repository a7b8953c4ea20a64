"""ctypes binding of the FP64 CPU oracle (oracle/lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark.  The product package never imports this module.

Arrays follow the C layout: populations [9][ny][nx], scalar fields [ny][nx],
x fastest, float64, C-contiguous.
"""
import ctypes
import os

import numpy as np

from . import build as _build

RC, RNR = 0, 1
PERIODIC, WALL, MOVING_WALL = 0, 1, 2
XMIN, XMAX, YMIN, YMAX = 0, 1, 2, 3

# Eq. 2 ordering of the velocity set (e_y = a * CY)
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("a", ctypes.c_double),
        ("cs2", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("omega", ctypes.c_double * 9),
        ("force", ctypes.c_double * 2),
        ("collision", ctypes.c_int),
        ("corrections", ctypes.c_int),
        ("bc_type", ctypes.c_int * 4),
        ("u_wall", (ctypes.c_double * 2) * 4),
        ("solid", ctypes.c_void_p),
    ]


def make_params(nx, ny, a, cs2, omega, force=(0.0, 0.0), rho0=1.0, collision=RC,
                corrections=True, bc=(PERIODIC,) * 4, u_wall=((0.0, 0.0),) * 4, solid=None):
    """solid: optional obstacle mask (ny, nx), nonzero = solid node."""
    p = Params()
    if solid is not None:
        m = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
        if m.shape != (int(ny), int(nx)):
            raise ValueError(f"mask shape {m.shape} != {(int(ny), int(nx))}")
        p._solid_keep = m  # the C side borrows this buffer
        p.solid = m.ctypes.data
    else:
        p.solid = None
    p.nx, p.ny, p.a, p.cs2, p.rho0 = int(nx), int(ny), float(a), float(cs2), float(rho0)
    for k in range(9):
        p.omega[k] = float(omega[k])
    p.force[0], p.force[1] = float(force[0]), float(force[1])
    p.collision = int(collision)
    p.corrections = 1 if corrections else 0
    for f in range(4):
        p.bc_type[f] = int(bc[f])
        p.u_wall[f][0] = float(u_wall[f][0])
        p.u_wall[f][1] = float(u_wall[f][1])
    return p


def paper_rates(tau, omega_bulk=1.0):
    """The paper's setting: omega_4 = omega_5 = 1/tau, omega_3 for the bulk
    viscosity, all other rates 1 (Sec. 2.2 and Sec. 5.1)."""
    w = [1.0] * 9
    w[3] = omega_bulk
    w[4] = w[5] = 1.0 / tau
    return w


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER(Params)
        sigs = {
            "orc_T": [ctypes.c_double, _D],
            "orc_Tinv": [ctypes.c_double, _D],
            "orc_F": [ctypes.c_double, ctypes.c_double, _D],
            "orc_macro": [P, _D, _D, _D, _D],
            "orc_feq": [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D],
            "orc_strain_rate": [P, _D, ctypes.c_double, ctypes.c_double, _D, _D],
            "orc_corrections": [P, _D, ctypes.c_double, ctypes.c_double, _D, _D],
            "orc_collide_node": [P, _D, ctypes.c_double, ctypes.c_double, _D],
            "orc_init": [P, _D, _D, _D, _D],
            "orc_density": [P, _D, _D],
            "orc_density_gradient": [P, _D, _D, _D],
            "orc_collide": [P, _D, _D],
            "orc_stream": [P, _D, _D],
            "orc_run": [P, _D, _D, ctypes.c_long],
            "orc_step_node": [P, _D, ctypes.c_int, ctypes.c_int, _D],
            "orc_moments": [P, _D, _D, _D, _D],
            "orc_stress": [P, _D, _D, _D, _D],
            "orc_set_threads": [ctypes.c_int],
        }
        for name, argtypes in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = argtypes
            fn.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(arr):
    if arr is None:
        return None
    assert arr.dtype == np.float64 and arr.flags["C_CONTIGUOUS"]
    return arr.ctypes.data_as(_D)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def T(a):
    out = np.zeros((9, 9))
    lib().orc_T(a, _ptr(out))
    return out


def Tinv(a):
    out = np.zeros((9, 9))
    lib().orc_Tinv(a, _ptr(out))
    return out


def F(ux, uy):
    out = np.zeros((9, 9))
    lib().orc_F(ux, uy, _ptr(out))
    return out


def macro(p, f9):
    f9 = _f64(f9)
    r, ux, uy = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_macro(ctypes.byref(p), _ptr(f9), ctypes.byref(r), ctypes.byref(ux), ctypes.byref(uy))
    return r.value, ux.value, uy.value


def feq(p, rho, ux, uy):
    out = np.zeros(9)
    lib().orc_feq(ctypes.byref(p), rho, ux, uy, _ptr(out))
    return out


def strain_rate(p, f9, gx, gy):
    f9 = _f64(f9)
    X, Y = ctypes.c_double(), ctypes.c_double()
    lib().orc_strain_rate(ctypes.byref(p), _ptr(f9), gx, gy, ctypes.byref(X), ctypes.byref(Y))
    return X.value, Y.value


def corrections(p, f9, gx, gy):
    f9 = _f64(f9)
    d3, d4 = ctypes.c_double(), ctypes.c_double()
    lib().orc_corrections(ctypes.byref(p), _ptr(f9), gx, gy, ctypes.byref(d3), ctypes.byref(d4))
    return d3.value, d4.value


def collide_node(p, f9, gx, gy):
    f9 = _f64(f9)
    out = np.zeros(9)
    lib().orc_collide_node(ctypes.byref(p), _ptr(f9), gx, gy, _ptr(out))
    return out


def init(p, rho=None, ux=None, uy=None):
    f = np.zeros((9, p.ny, p.nx))
    args = [None if v is None else _f64(v) for v in (rho, ux, uy)]
    lib().orc_init(ctypes.byref(p), *[_ptr(v) for v in args], _ptr(f))
    return f


def density(p, f):
    f = _f64(f)
    rho = np.zeros((p.ny, p.nx))
    lib().orc_density(ctypes.byref(p), _ptr(f), _ptr(rho))
    return rho


def density_gradient(p, rho):
    rho = _f64(rho)
    gx = np.zeros((p.ny, p.nx))
    gy = np.zeros((p.ny, p.nx))
    lib().orc_density_gradient(ctypes.byref(p), _ptr(rho), _ptr(gx), _ptr(gy))
    return gx, gy


def collide(p, f):
    f = _f64(f)
    ft = np.zeros_like(f)
    lib().orc_collide(ctypes.byref(p), _ptr(f), _ptr(ft))
    return ft


def stream(p, ft):
    ft = _f64(ft)
    f = np.zeros_like(ft)
    lib().orc_stream(ctypes.byref(p), _ptr(ft), _ptr(f))
    return f


def run(p, f, nsteps):
    """Advance f (a copy) by nsteps collide+stream steps and return it."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    lib().orc_run(ctypes.byref(p), _ptr(f), None, int(nsteps))
    return f


def step_node(p, f, i, j):
    """Populations of node (i, j) after one step, from the whole field f."""
    f = _f64(f)
    out = np.zeros(9)
    lib().orc_step_node(ctypes.byref(p), _ptr(f), int(i), int(j), _ptr(out))
    return out


def moments(p, f):
    f = _f64(f)
    rho = np.zeros((p.ny, p.nx))
    ux = np.zeros((p.ny, p.nx))
    uy = np.zeros((p.ny, p.nx))
    lib().orc_moments(ctypes.byref(p), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


def set_threads(n):
    lib().orc_set_threads(int(n))


def max_threads():
    return lib().orc_max_threads()


def stress(p, f):
    """Local viscous stress (tau_xx, tau_yy, tau_xy), each (ny, nx)."""
    f = _f64(f)
    out = [np.zeros((p.ny, p.nx)) for _ in range(3)]
    lib().orc_stress(ctypes.byref(p), _ptr(f), *[_ptr(o) for o in out])
    return tuple(out)

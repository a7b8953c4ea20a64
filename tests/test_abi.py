"""The C ABI library loads and exports every entry point include/lbm.h and
include/lbm_batch.h declare; host-side argument validation works without a
GPU (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2103_02119_amd import lbm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
BATCH_HEADER = os.path.join(ROOT, "include", "lbm_batch.h")
NN_HEADER = os.path.join(ROOT, "include", "lbm_nn.h")


def _declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("lbm_create", "lbm_step", "lbm_moments", "lbm_residual", "lbm_sums",
                     "lbm_set_fields", "lbm_get_populations", "lbm_set_populations",
                     "lbm_destroy", "lbm_last_error", "lbm_required_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in (_declared_functions() + _declared_functions(BATCH_HEADER)
                 + _declared_functions(NN_HEADER)):
        assert hasattr(lib, name), name


def test_binding_uses_the_same_names():
    assert sorted(L.EXPORTS) == _declared_functions()
    assert sorted(L.BATCH_EXPORTS) == _declared_functions(BATCH_HEADER)
    for name in L.EXPORTS + L.BATCH_EXPORTS:
        assert callable(getattr(L, name))
    from paper_2103_02119_amd import nn as K
    assert sorted(K.EXPORTS) == _declared_functions(NN_HEADER)
    for name in K.EXPORTS:
        assert callable(getattr(K, name))


def test_nn_rejects_bad_shapes_before_touching_the_device():
    from paper_2103_02119_amd import nn as K
    lib = K.load()
    # channels not a multiple of 8, odd pooled size, missing pointers
    assert lib.lbm_nn_conv3x3_fwd(1, 12, None, 0, 1, 8, 8, 1, 1, 32, 1, 1, None) == -1
    assert lib.lbm_nn_conv3x3_fwd(1, 16, None, 8, 1, 8, 8, 1, 1, 32, 1, 1, None) == -1
    assert lib.lbm_nn_conv3x3_dgrad(1, 1, 8, 8, 30, 1, 1, 16, None, 0, 0, None) == -1
    assert lib.lbm_nn_avgpool2_fwd(1, 1, 7, 8, 4, 1, None) == -1
    assert lib.lbm_nn_conv3x3_wgrad(1, 16, None, 0, 1, 8, 8, 1, 32, 1, 1, 1, 0, None) == -1
    assert lib.lbm_nn_adam(1, 1, 1, 1, 10, 0.1, 0.9, 0.99, 1e-8, 0, None) == -1


def test_required_bytes():
    assert L.lbm_required_bytes(512, 1024, L.LBM_FP32_DEV) == 9 * 512 * 1024 * 4
    assert L.lbm_required_bytes(100, 10, L.LBM_FP64) == 9 * 128 * 10 * 8
    assert L.lbm_required_bytes(3, 3, L.LBM_FP64_DEV) == 9 * 64 * 3 * 8
    with pytest.raises(L.LbmError) as e:
        L.lbm_required_bytes(2, 10, L.LBM_FP64)
    assert e.value.code == L.LBM_E_INVAL
    with pytest.raises(L.LbmError):
        L.lbm_required_bytes(10, 10, 7)
    with pytest.raises(L.LbmError):
        L.lbm_required_bytes(1 << 16, 1 << 16, L.LBM_FP64)


def _bc(types=(0, 0, 1, 1)):
    return L.make_bc(types)


@pytest.mark.parametrize("kwargs,fragment", [
    (dict(nx=2), "nx and ny"),
    (dict(r=0.0), "r must be"),
    (dict(r=-1.0), "r must be"),
    (dict(rates=[1.0] * 8 + [2.0]), "rates[8]"),
    (dict(rates=[0.0] + [1.0] * 8), "rates[0]"),
    (dict(cs2=0.25), "cs2"),
    (dict(cs2=-0.1), "cs2"),
    (dict(bc=(0, 1, 1, 1)), "opposite faces"),
    (dict(bc=(0, 0, 1, 5)), "unknown boundary"),
    (dict(collision=3), "unknown collision"),
    (dict(precision=9), "unknown precision"),
    (dict(rows_per_wave=65), "rows_per_wave"),
])
def test_invalid_arguments_are_rejected_before_touching_the_device(kwargs, fragment):
    args = dict(nx=32, ny=16, r=0.5, rates=[1.0] * 9, bc=(0, 0, 1, 1), cs2=0.16, collision=0,
                precision=0, rows_per_wave=0)
    args.update(kwargs)
    o = L.lbm_default_opts()
    o.cs2 = args["cs2"]
    o.collision = args["collision"]
    o.precision = args["precision"]
    o.rows_per_wave = args["rows_per_wave"]
    with pytest.raises(L.LbmError) as e:
        L.lbm_create(args["nx"], args["ny"], args["r"], args["rates"], _bc(args["bc"]), o)
    assert e.value.code == L.LBM_E_INVAL
    assert fragment in str(e.value)
    assert fragment in L.lbm_last_error(None)


def test_caller_buffers_must_be_paired_and_large_enough():
    o = L.lbm_default_opts()
    o.f_a = 0x1000
    with pytest.raises(L.LbmError) as e:
        L.lbm_create(32, 16, 0.5, [1.0] * 9, _bc(), o)
    assert e.value.code == L.LBM_E_INVAL
    o.f_b = 0x2000
    o.f_bytes = 16
    with pytest.raises(L.LbmError) as e:
        L.lbm_create(32, 16, 0.5, [1.0] * 9, _bc(), o)
    assert e.value.code == L.LBM_E_INVAL


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU driver is present")
def test_no_gpu_fails_loudly():
    with pytest.raises(L.LbmError) as e:
        L.lbm_create(32, 16, 0.5, [1.0] * 9, _bc())
    assert e.value.code == L.LBM_E_DEVICE


def test_default_opts():
    o = L.lbm_default_opts()
    assert o.rho0 == 1.0 and o.collision == L.LBM_RC and o.precision == L.LBM_FP64
    assert o.corrections == 1 and o.cs2 == 0.0 and o.stream is None


# ---------------------------------------------------------------- batches

def _case(**kw):
    args = dict(nx=32, ny=16, r=0.5, rates=[1.0] * 9, bc_types=(0, 0, 1, 1), cs2=0.16)
    args.update(kw)
    return L.make_case(**args)


@pytest.mark.parametrize("bad,fragment", [
    (dict(nx=2), "case 1: nx and ny"),
    (dict(r=0.0), "case 1: r must be"),
    (dict(rates=[1.0] * 8 + [2.0]), "case 1: rates[8]"),
    (dict(cs2=0.3), "case 1: cs2"),
    (dict(bc_types=(0, 1, 1, 1)), "case 1: opposite faces"),
])
def test_batch_rejects_a_bad_case_with_its_index(bad, fragment):
    with pytest.raises(L.LbmError) as e:
        L.lbm_batch_create([_case(), _case(**bad)])
    assert e.value.code == L.LBM_E_INVAL
    assert fragment in str(e.value)
    assert fragment in L.lbm_batch_last_error(None)


@pytest.mark.parametrize("field,value,fragment", [
    ("collision", 2, "unknown collision"),
    ("precision", 4, "unknown precision"),
    ("rows_per_wave", 65, "rows_per_wave"),
    ("workgroups", -1, "workgroups"),
    ("graph_steps", 3, "graph_steps"),
])
def test_batch_rejects_bad_options(field, value, fragment):
    o = L.lbm_batch_default_opts()
    setattr(o, field, value)
    with pytest.raises(L.LbmError) as e:
        L.lbm_batch_create([_case()], o)
    assert e.value.code == L.LBM_E_INVAL and fragment in str(e.value)


def test_batch_needs_a_case():
    with pytest.raises(L.LbmError) as e:
        L.lbm_batch_create([])
    assert e.value.code == L.LBM_E_INVAL


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU driver is present")
def test_batch_without_gpu_fails_loudly():
    with pytest.raises(L.LbmError) as e:
        L.lbm_batch_create([_case()])
    assert e.value.code == L.LBM_E_DEVICE


def test_batch_default_opts():
    o = L.lbm_batch_default_opts()
    assert o.collision == L.LBM_RC and o.precision == L.LBM_FP64 and o.corrections == 1
    assert o.rows_per_wave == 0 and o.workgroups == 0 and o.graph_steps == 0 and o.stream is None


def test_null_handles_are_rejected_before_touching_the_device():
    lib = L.load()
    D = ctypes.POINTER(ctypes.c_double)
    d = (ctypes.c_double * 9)()
    pd = ctypes.cast(d, D)
    calls = {
        "lbm_set_fields": (None, None, None, None),
        "lbm_step": (None, 1),
        "lbm_moments": (None, None, None, None),
        "lbm_stress": (None, None, None, None),
        "lbm_sums": (None, pd),
        "lbm_residual": (None, pd),
        "lbm_check_async": (None,),
        "lbm_check_result": (None, pd, pd, None),
        "lbm_get_populations": (None, pd),
        "lbm_set_populations": (None, pd),
        "lbm_set_mask": (None, None),
        "lbm_set_rates": (None, pd),
        "lbm_set_force": (None, 0.0, 0.0),
        "lbm_step_forced": (None, 1, pd, pd),
        "lbm_smooth_step": (None,),
        "lbm_set_steps_per_launch": (None, 1),
        "lbm_set_two_step_form": (None, 1),
        "lbm_check_into": (None, None),
    }
    for name, args in calls.items():
        assert getattr(lib, name)(*args) == L.LBM_E_INVAL, name
    assert lib.lbm_steps_per_launch(None) == L.LBM_E_INVAL
    assert lib.lbm_two_step_form(None) == L.LBM_E_INVAL
    assert lib.lbm_destroy(None) == L.LBM_OK
    assert lib.lbm_batch_step(None, 1) == L.LBM_E_INVAL
    assert lib.lbm_batch_destroy(None) == L.LBM_OK
    assert lib.lbm_batch_steps_per_launch(None) == L.LBM_E_INVAL
    assert lib.lbm_batch_two_step_form(None) == L.LBM_E_INVAL


def test_stream_copy_validates_before_touching_the_device():
    lib = L.load()
    assert lib.lbm_stream_copy(None, ctypes.c_void_p(0x1000), 16, 0, None) == L.LBM_E_INVAL
    assert lib.lbm_stream_copy(ctypes.c_void_p(0x1000), None, 16, 0, None) == L.LBM_E_INVAL
    # sizes and addresses must be multiples of 16 bytes
    assert lib.lbm_stream_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 24, 0,
                               None) == L.LBM_E_INVAL
    assert lib.lbm_stream_copy(ctypes.c_void_p(0x1008), ctypes.c_void_p(0x2000), 32, 0,
                               None) == L.LBM_E_INVAL
    assert lib.lbm_stream_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 32, -1,
                               None) == L.LBM_E_INVAL
    assert "16 bytes" in L.lbm_last_error(None) or "workgroups" in L.lbm_last_error(None)

"""Host-side checks of the C ABI library (no GPU needed): it was built for
gfx950, it loads, and it exports every entry point that include/nbody.h
declares, with the documented status codes and enum values."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2605_02744_amd as nb
    if not os.path.exists(nb.LIB_PATH):
        pytest.fail("libnbody_accel.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(nb.LIB_PATH)


def test_header_declares_expected_calls():
    names = _declared()
    for required in ("nbody_accel", "nbody_step", "nbody_energy", "nbody_step_batched",
                     "nbody_accel_vjp", "nbody_traj_grad", "nbody_last_error", "nbody_tune"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_library_targets_gfx950():
    """The embedded device code object names the gfx950 target."""
    import paper_2605_02744_amd as nb
    data = open(nb.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_version_and_error_without_gpu_call(lib):
    lib.nbody_version.restype = ctypes.c_int
    assert lib.nbody_version() >= 100
    lib.nbody_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.nbody_last_error(), bytes)


def test_status_and_enum_values_match_header():
    import paper_2605_02744_amd as nb
    text = open(HEADER).read()
    for name in ("NBODY_OK", "NBODY_EINVAL", "NBODY_EHIP", "NBODY_ENOMEM", "NBODY_ENONFINITE",
                 "NBODY_EUNSUPPORTED", "NBODY_FP64", "NBODY_FP32C", "NBODY_FP32",
                 "NBODY_EXCLUDE_SELF", "NBODY_CHECK_FINITE", "NBODY_ACC_VALID"):
        mm = re.search(r"\b%s\s*=\s*(-?\d+)" % name, text)
        assert mm, name
        assert getattr(nb, name) == int(mm.group(1)), name


def test_invalid_arguments_rejected_before_any_gpu_work(lib):
    """Argument checks that need no device: NULL params, negative n, bad flags."""
    import paper_2605_02744_amd as nb
    from paper_2605_02744_amd._binding import nbody_params
    L = nb.load()
    assert L.nbody_accel(10, None, None, None, None, None) == nb.NBODY_EINVAL
    p = nbody_params(1.0, 0.01, nb.NBODY_FP32C, 0)
    assert L.nbody_accel(-1, None, None, None, ctypes.byref(p), None) == nb.NBODY_EINVAL
    assert b"n < 0" in L.nbody_last_error()
    bad = nbody_params(1.0, -0.5, nb.NBODY_FP32C, 0)
    assert L.nbody_accel(0, None, None, None, ctypes.byref(bad), None) == nb.NBODY_EINVAL
    zero = nbody_params(1.0, 0.0, nb.NBODY_FP32C, 0)
    assert L.nbody_accel(0, None, None, None, ctypes.byref(zero), None) == nb.NBODY_EINVAL
    assert b"EXCLUDE_SELF" in L.nbody_last_error()
    prec = nbody_params(1.0, 0.1, 7, 0)
    assert L.nbody_accel(0, None, None, None, ctypes.byref(prec), None) == nb.NBODY_EINVAL
    flg = nbody_params(1.0, 0.1, 0, 1 << 9)
    assert L.nbody_accel(0, None, None, None, ctypes.byref(flg), None) == nb.NBODY_EINVAL
    nanG = nbody_params(float("nan"), 0.1, 0, 0)
    assert L.nbody_accel(0, None, None, None, ctypes.byref(nanG), None) == nb.NBODY_EINVAL
    assert L.nbody_step(0, None, None, None, None, float("inf"), 1, ctypes.byref(p), None) == nb.NBODY_EINVAL
    assert L.nbody_step(0, None, None, None, None, 0.1, -1, ctypes.byref(p), None) == nb.NBODY_EINVAL
    assert L.nbody_traj_grad(0, None, None, 0, 5, None, 0.1, None, None, None, None, None,
                             ctypes.byref(p), None) == nb.NBODY_EINVAL
    # n == 0 is a documented no-op
    assert L.nbody_accel(0, None, None, None, ctypes.byref(p), None) == nb.NBODY_OK


def test_batched_host_validation(lib):
    import numpy as np
    import paper_2605_02744_amd as nb
    from paper_2605_02744_amd._binding import nbody_params
    L = nb.load()
    p = nbody_params(1.0, 0.0, nb.NBODY_FP32C, 0)
    off = np.array([0, 5, 3], dtype=np.int64)
    eps = np.array([0.1, 0.1])
    PI = ctypes.POINTER(ctypes.c_int64)
    PD = ctypes.POINTER(ctypes.c_double)
    st = L.nbody_step_batched(2, off.ctypes.data_as(PI), eps.ctypes.data_as(PD), None, None, None, None,
                              0.1, 1, ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL and b"non-decreasing" in L.nbody_last_error()
    off = np.array([1, 5, 9], dtype=np.int64)
    st = L.nbody_step_batched(2, off.ctypes.data_as(PI), eps.ctypes.data_as(PD), None, None, None, None,
                              0.1, 1, ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL
    off = np.array([0, 5, 9], dtype=np.int64)
    eps0 = np.array([0.1, 0.0])
    st = L.nbody_step_batched(2, off.ctypes.data_as(PI), eps0.ctypes.data_as(PD), None, None, None, None,
                              0.1, 1, ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL


def test_tune_batched_host_validation(lib):
    import numpy as np
    import paper_2605_02744_amd as nb
    from paper_2605_02744_amd._binding import nbody_params
    L = nb.load()
    p = nbody_params(1.0, 0.0, nb.NBODY_FP32C, 0)
    PI = ctypes.POINTER(ctypes.c_int64)
    PD = ctypes.POINTER(ctypes.c_double)
    off = np.array([0, 0], dtype=np.int64)
    eps = np.array([0.1])
    st = L.nbody_tune_batched(1, off.ctypes.data_as(PI), eps.ctypes.data_as(PD), None, None, None, 0.1, 4, 1,
                              ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL and b"empty" in L.nbody_last_error()
    off = np.array([0, 10], dtype=np.int64)
    st = L.nbody_tune_batched(1, off.ctypes.data_as(PI), eps.ctypes.data_as(PD), None, None, None, 0.1, 0, 1,
                              ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL and b"nsteps" in L.nbody_last_error()
    st = L.nbody_tune_batched(1, off.ctypes.data_as(PI), eps.ctypes.data_as(PD), None, None, None, 0.1, 4, 3,
                              ctypes.byref(p), None)
    assert st == nb.NBODY_EINVAL and b"allow_cooperative" in L.nbody_last_error()


def test_set_config_validation(lib):
    import paper_2605_02744_amd as nb
    with pytest.raises(nb.NBodyError):
        nb.nbody_set_config(ipl=3)
    with pytest.raises(nb.NBodyError):
        nb.nbody_set_config(split=5000)
    with pytest.raises(nb.NBodyError):
        nb.nbody_set_config(bsplit=5)
    with pytest.raises(nb.NBodyError):
        nb.nbody_set_config(bpass=3)
    with pytest.raises(nb.NBodyError):
        nb.nbody_set_config(bitem=300)
    with pytest.raises(nb.NBodyError):
        nb.nbody_set_config(bitem=32)
    with pytest.raises(nb.NBodyError):
        nb.nbody_set_config(sweep=2)
    nb.nbody_set_config(bsplit=2, bitem=64)
    nb.nbody_set_config(bsplit=4)
    nb.nbody_set_config(ipl=2, split=4)
    nb.nbody_set_config(sweep=1)
    nb.nbody_set_config()


def _header_struct_fields(name):
    """(type, field) pairs of `typedef struct name { ... } name;` in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, flags=re.S).group(1)
    return re.findall(r"\b(int32_t|uint32_t|double)\s+(\w+)\s*;", body)


def test_binding_structs_match_header():
    """The ctypes structures of the binding have the header's fields, in the
    header's order and types (a drift would silently shift every later field)."""
    import ctypes as ct
    from paper_2605_02744_amd import _binding as B
    ctype = {"int32_t": ct.c_int32, "uint32_t": ct.c_uint32, "double": ct.c_double}
    for name, cls in (("nbody_config", B.nbody_config), ("nbody_params", B.nbody_params)):
        fields = _header_struct_fields(name)
        assert fields, name
        assert [(f, ctype[t]) for t, f in fields] == [(f, t) for f, t in cls._fields_], name

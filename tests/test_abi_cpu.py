"""Host-side checks of the C ABI: the library loads, exports every function
include/csmri.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1203_4587_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "csmri.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_[a-z_A-Z0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libcsmri.so is not built (run python -m paper_1203_4587_amd.build)")
    return _lib.load()


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert "cs_admm_solve" in names and "cs_plan_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTED) == names


def test_status_strings(lib):
    for st in range(6):
        assert lib.cs_status_string(st)
    assert b"unknown" in lib.cs_status_string(99)
    assert lib.cs_version() >= 10000


def _desc(nv=64, nh=64, nt=8, nc=4, prior=0, rho=0.5):
    return _lib.CsPlanDesc(nv, nh, nt, nc, prior, rho, 0)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced on the paths below


def _create(lib, desc, mu=0.1, alloc=None, coil=FAKE, mask=FAKE):
    h = ctypes.c_void_p()
    st = lib.cs_plan_create(ctypes.byref(desc) if desc is not None else None, coil, mask, mu,
                            ctypes.byref(alloc) if alloc is not None else None, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw,expect", [
    (dict(nv=1), _lib.CS_EINVAL),
    (dict(nc=0), _lib.CS_EINVAL),
    (dict(nt=1, prior=0), _lib.CS_EINVAL),          # TV needs two frames
    (dict(prior=7), _lib.CS_EINVAL),
    (dict(rho=0.0), _lib.CS_EINVAL),
    (dict(nv=100), _lib.CS_EUNSUPPORTED),           # not 2^a 3^b
    (dict(nh=1024), _lib.CS_EUNSUPPORTED),          # > 512
    (dict(nt=65), _lib.CS_EUNSUPPORTED),
    (dict(nc=65), _lib.CS_EUNSUPPORTED),
])
def test_plan_create_rejects_bad_descriptors(lib, kw, expect):
    st, h = _create(lib, _desc(**kw))
    assert st == expect, lib.cs_last_error()
    assert h.value is None
    assert lib.cs_last_error()


def test_plan_create_rejects_bad_scalars_and_nulls(lib):
    assert _create(lib, _desc(), mu=0.0)[0] == _lib.CS_EINVAL
    assert _create(lib, _desc(), mu=float("nan"))[0] == _lib.CS_EINVAL
    assert _create(lib, None)[0] == _lib.CS_EINVAL
    assert _create(lib, _desc(), coil=None)[0] == _lib.CS_EINVAL
    assert lib.cs_plan_create(ctypes.byref(_desc()), FAKE, FAKE, 0.1, None, None, None) == _lib.CS_EINVAL


def test_allocator_failure_is_enomem(lib):
    calls = []

    def alloc(nbytes, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, ctx):
        raise AssertionError("nothing was allocated")
    a = _lib.CsAllocator(_lib.ALLOC_FN(alloc), _lib.FREE_FN(free), None)
    st, h = _create(lib, _desc(nv=256, nh=256, nt=32, nc=8), alloc=a)
    assert st == _lib.CS_ENOMEM
    assert h.value is None
    # the first request is the packed factor: nh*nt blocks of nv(nv+1)/2 complex64
    assert calls and calls[0] >= 256 * 32 * (256 * 257 // 2) * 8


def test_eigen_plan_asks_first_for_both_eigenvector_copies(lib):
    """With CS_FLAG_EIGEN the first (largest) request is U stored twice
    instead of the packed inverse; a NULL from the allocator is CS_ENOMEM."""
    calls = []

    def alloc(nbytes, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, ctx):
        raise AssertionError("nothing was allocated")
    a = _lib.CsAllocator(_lib.ALLOC_FN(alloc), _lib.FREE_FN(free), None)
    d = _desc(nv=256, nh=256, nt=32, nc=8)
    d.flags = _lib.CS_FLAG_EIGEN
    st, h = _create(lib, d, alloc=a)
    assert st == _lib.CS_ENOMEM and h.value is None
    assert calls == [256 * 32 * 256 * 256 * 8]


def test_header_flag_values_match_the_binding():
    text = open(os.path.join(ROOT, "include", "csmri.h")).read()
    found = dict(re.findall(r"\b(CS_FLAG_[A-Z_]+)\s*=\s*1u\s*<<\s*(\d+)", text))
    assert "CS_FLAG_CHECK_FINITE" in found and len(found) == 7
    for name, bit in found.items():
        assert getattr(_lib, name) == 1 << int(bit), name


def test_null_plan_calls_are_einval(lib):
    assert lib.cs_apply_A(None, FAKE, FAKE, None) == _lib.CS_EINVAL
    assert lib.cs_apply_AH(None, FAKE, FAKE, None) == _lib.CS_EINVAL
    assert lib.cs_apply_block_inverse(None, FAKE, FAKE, None) == _lib.CS_EINVAL
    assert lib.cs_admm_solve(None, FAKE, 0.01, 0.1, 10, FAKE, None, None, None) == _lib.CS_EINVAL
    assert lib.cs_plan_destroy(None) == _lib.CS_OK
    n = ctypes.c_size_t()
    assert lib.cs_plan_bytes(None, ctypes.byref(n)) == _lib.CS_EINVAL


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()


@pytest.mark.parametrize("flags", [
    _lib.CS_FLAG_XU_WAVE | _lib.CS_FLAG_XU_GROUP,   # exclusive x-update forms
    1 << 12,                                        # unknown bit
])
def test_plan_create_rejects_bad_flags(lib, flags):
    d = _desc()
    d.flags = flags
    st, h = _create(lib, d)
    assert st == _lib.CS_EINVAL
    assert h.value is None


def test_flag_and_tune_calls_reject_nulls(lib):
    f = ctypes.c_uint32()
    assert lib.cs_plan_flags(None, ctypes.byref(f)) == _lib.CS_EINVAL
    assert lib.cs_plan_set_flags(None, 0) == _lib.CS_EINVAL
    assert lib.cs_plan_tune(None, FAKE, 0.01, 5, None, 0, None, None) == _lib.CS_EINVAL


def test_batch_calls_reject_bad_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.cs_batch_create(None, 1, None, None, ctypes.byref(h)) == _lib.CS_EINVAL
    sl = (_lib.CsSliceDesc * 2)()
    sl[0] = _lib.CsSliceDesc(_desc(), FAKE.value, FAKE.value, 0.1)
    sl[1] = _lib.CsSliceDesc(_desc(), FAKE.value, FAKE.value, 0.1)
    assert lib.cs_batch_create(sl, 0, None, None, ctypes.byref(h)) == _lib.CS_EINVAL
    assert lib.cs_batch_create(sl, 2, None, None, None) == _lib.CS_EINVAL
    # a bad descriptor fails the whole batch before any device work, naming the slice
    sl[0] = _lib.CsSliceDesc(_desc(nv=100), FAKE.value, FAKE.value, 0.1)
    assert lib.cs_batch_create(sl, 2, None, None, ctypes.byref(h)) == _lib.CS_EUNSUPPORTED
    assert h.value is None
    assert b"slice 0" in lib.cs_last_error()
    n = ctypes.c_int32()
    p = ctypes.c_void_p()
    assert lib.cs_batch_size(None, ctypes.byref(n)) == _lib.CS_EINVAL
    assert lib.cs_batch_plan(None, 0, ctypes.byref(p)) == _lib.CS_EINVAL
    assert lib.cs_batch_solve(None, None, None, 10, None, None) == _lib.CS_EINVAL
    assert lib.cs_batch_destroy(None) == _lib.CS_OK


def test_gradient_calls_reject_bad_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.cs_grad_create(None, 20, 5, ctypes.byref(h)) == _lib.CS_EINVAL
    assert lib.cs_grad_create(FAKE, 20, 5, None) == _lib.CS_EINVAL
    assert lib.cs_admm_forward_ckpt(None, FAKE, 0.01, 0.1, FAKE, None) == _lib.CS_EINVAL
    assert lib.cs_admm_backward(None, FAKE, FAKE, FAKE, None) == _lib.CS_EINVAL
    assert lib.cs_grad_destroy(None) == _lib.CS_OK


def test_delta_solve_rejects_bad_arguments(lib):
    n = ctypes.c_int32()
    d = ctypes.c_float()
    assert lib.cs_admm_solve_until(None, FAKE, 0.01, 0.1, 10, 1e-3, 5, FAKE, None, ctypes.byref(n),
                                   ctypes.byref(d), None) == _lib.CS_EINVAL
    assert lib.cs_admm_solve_until(FAKE, FAKE, 0.01, 0.1, 10, 1e-3, 5, FAKE, None, None, None,
                                   None) == _lib.CS_EINVAL
    assert lib.cs_admm_solve_until(FAKE, FAKE, 0.01, 0.1, 0, 1e-3, 5, FAKE, None, ctypes.byref(n), None,
                                   None) == _lib.CS_EINVAL
    assert lib.cs_admm_solve_until(FAKE, FAKE, 0.01, 0.1, 10, 1e-3, 0, FAKE, None, ctypes.byref(n), None,
                                   None) == _lib.CS_EINVAL
    assert lib.cs_admm_solve_until(FAKE, FAKE, 0.01, 0.1, 10, float("nan"), 5, FAKE, None, ctypes.byref(n), None,
                                   None) == _lib.CS_EINVAL


def test_fft_tile_calls_reject_bad_arguments(lib):
    c, r = ctypes.c_int32(), ctypes.c_int32()
    assert lib.cs_plan_fft_tiles(None, ctypes.byref(c), ctypes.byref(r)) == _lib.CS_EINVAL
    assert lib.cs_plan_set_fft_tiles(None, 4, 4) == _lib.CS_EINVAL


def test_read_stream_rejects_bad_arguments(lib):
    sink = ctypes.c_void_p(0x2000)
    assert lib.cs_read_stream(None, 1 << 20, 0, sink, None) == _lib.CS_EINVAL
    assert lib.cs_read_stream(FAKE, 1 << 20, 0, None, None) == _lib.CS_EINVAL
    assert lib.cs_read_stream(FAKE, 0, 0, sink, None) == _lib.CS_EINVAL
    assert lib.cs_read_stream(FAKE, 24, 0, sink, None) == _lib.CS_EINVAL       # not a multiple of 16
    assert lib.cs_read_stream(ctypes.c_void_p(0x1008), 32, 0, sink, None) == _lib.CS_EINVAL  # misaligned
    assert lib.cs_read_stream(FAKE, 32, -1, sink, None) == _lib.CS_EINVAL
    assert lib.cs_read_stream(FAKE, 32, 65536, sink, None) == _lib.CS_EINVAL

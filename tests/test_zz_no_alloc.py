"""cs_apply_AH_noalloc, the plan-free H'y that allocates nothing: through
the C ABI, its output equals cs_apply_AH of a plan built on the same coil
maps and mask (relative l2 within 1e-6, elementwise within 1e-5 of the
largest value), on consecutive calls that share the library's device array --
a second, smaller call after a larger one, and a call that needs several
frame chunks -- and sizes beyond the array are refused."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1203_4587_amd import _lib
from tests.helpers import make_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _noalloc(coil, mask, y, out):
    lib = _lib.load()
    nc, nv, nh = coil.shape
    nt = mask.shape[0]
    d = _lib.CsPlanDesc(nv, nh, nt, nc, 0, 0.5, 0)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    return lib.cs_apply_AH_noalloc(ctypes.byref(d), p(coil), p(mask), p(y), p(out),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _check(case):
    from paper_1203_4587_amd.api import Plan
    coil, mask, y = case.device()
    ref = Plan(coil, mask, 0.1, prior="tv" if case.mask.shape[0] > 1 else "dft").apply_AH(y)
    out = torch.full_like(ref, complex(float("nan"), 0.0))
    st = _noalloc(coil, mask, y, out)
    assert st == _lib.CS_OK, _lib.load().cs_last_error()
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    assert np.isfinite(a).all()
    err = rel_l2(a, b)
    print(case.mask.shape, coil.shape, "rel_l2 vs cs_apply_AH", err, "bit-identical", bool((a == b).all()))
    assert err < 1e-6
    assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()
    # and the oracle's H'y
    assert rel_l2(a, O.adjoint(case.y, case.coil, case.mask)) < 1e-5
    return out


def test_noalloc_adjoint_equals_plan_adjoint_on_consecutive_calls():
    big = make_case(64, 48, 8, 4, accel=3, ncenter=4, seed=31)
    small = make_case(32, 24, 5, 3, accel=4, ncenter=2, seed=32)
    _check(big)
    _check(small)           # smaller call after a larger one: stale contents must not leak
    _check(big)


def test_noalloc_adjoint_in_frame_chunks_and_odd_sizes():
    # 256x256 with 16 coils: the array holds 6 of the 10 frames at once
    _check(make_case(256, 256, 10, 16, accel=8, ncenter=12, seed=33))
    _check(make_case(27, 12, 3, 2, accel=3, ncenter=2, seed=34))     # radix-3 sizes
    _check(make_case(384, 8, 2, 2, accel=4, ncenter=4, seed=35))     # 512-value wave groups
    e = make_case(16, 8, 3, 2, accel=2, ncenter=2, seed=36)
    e.mask[1] = 0                                                    # a frame with no sampled row
    e.y = e.y * e.mask[:, None, :, None]
    _check(e)


def test_noalloc_adjoint_allocates_nothing_and_refuses_oversize():
    case = make_case(64, 48, 8, 4, accel=3, ncenter=4, seed=37)
    coil, mask, y = case.device()
    out = torch.empty((8, 64, 48), dtype=torch.complex64, device="cuda")
    assert _noalloc(coil, mask, y, out) == _lib.CS_OK
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        assert _noalloc(coil, mask, y, out) == _lib.CS_OK
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    # 512 x 512 maps with 40 coils need 84 MB for the maps alone
    lib = _lib.load()
    d = _lib.CsPlanDesc(512, 512, 2, 40, 0, 0.5, 0)
    f = ctypes.c_void_p(out.data_ptr())
    assert lib.cs_apply_AH_noalloc(ctypes.byref(d), f, f, f, f, None) == _lib.CS_EUNSUPPORTED
    assert b"device array" in lib.cs_last_error()
    d = _lib.CsPlanDesc(100, 512, 2, 4, 0, 0.5, 0)
    assert lib.cs_apply_AH_noalloc(ctypes.byref(d), f, f, f, f, None) == _lib.CS_EUNSUPPORTED
    assert lib.cs_apply_AH_noalloc(None, f, f, f, f, None) == _lib.CS_EINVAL

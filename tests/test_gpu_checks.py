"""Input checks and allocation ownership on the GPU, through the C ABI:
CS_FLAG_CHECK_FINITE rejects NaN and infinity in the inputs each entry point
reads (and only there), and a CS_FLAG_EIGEN plan takes every device buffer of
its build, the eigensolver library's own workspace included, from the
caller's allocator."""
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


def _plan(case, prior="tv", flags=_lib.CS_FLAG_CHECK_FINITE):
    from paper_1203_4587_amd.api import Plan
    coil, mask, y = case.device()
    return Plan(coil, mask, 0.1, prior=prior, flags=flags), coil, mask, y


def _einval(fn, *args, **kw):
    with pytest.raises(RuntimeError, match="CS_EINVAL") as ei:
        fn(*args, **kw)
    assert "non-finite" in str(ei.value)


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_check_finite_rejects_sampled_kspace(bad):
    case = make_case(32, 16, 6, 3, seed=3)
    plan, coil, mask, y = _plan(case)
    ref = plan.solve(y, 0.01, 5)
    t, c = 2, 1
    ky = int(np.nonzero(case.mask[t])[0][1])
    yb = y.clone()
    yb[t, c, ky, 5] = complex(bad, 0.0)
    _einval(plan.solve, yb, 0.01, 5)
    _einval(plan.apply_AH, yb)
    _einval(plan.solve_until, yb, 0.01, 20)
    # the plan stays usable and unchanged
    assert torch.equal(plan.solve(y, 0.01, 5), ref)


def test_check_finite_ignores_unsampled_rows():
    case = make_case(32, 16, 6, 3, seed=4)
    plan, coil, mask, y = _plan(case)
    ref = plan.solve(y, 0.01, 5)
    t = 1
    ky = int(np.nonzero(case.mask[t] == 0)[0][0])
    yb = y.clone()
    yb[t, :, ky, :] = float("nan")
    assert torch.equal(plan.solve(yb, 0.01, 5), ref)
    xo = O.solve(case.y, case.coil, case.mask, "tv", 0.01, 0.1, 0.5, 5)["x"]
    assert rel_l2(ref.cpu().numpy(), xo) < 1e-4


def test_check_finite_images_and_coils():
    from paper_1203_4587_amd.api import Plan
    case = make_case(32, 16, 6, 3, seed=5)
    plan, coil, mask, y = _plan(case)
    x = plan.apply_AH(y)
    xb = x.clone()
    xb[3, 7, 2] = complex(0.0, float("nan"))
    _einval(plan.apply_A, xb)
    _einval(plan.block_inverse, xb)
    cb = coil.clone()
    cb[1, 4, 4] = float("inf")
    _einval(Plan, cb, mask, 0.1, prior="tv", flags=_lib.CS_FLAG_CHECK_FINITE)
    # without the flag the same calls run (the values are the caller's business)
    Plan(cb, mask, 0.1, prior="tv").close()
    # checked calls equal unchecked ones
    plain = Plan(coil, mask, 0.1, prior="tv")
    assert torch.equal(plan.apply_A(x), plain.apply_A(x))
    assert torch.equal(plan.apply_AH(y), plain.apply_AH(y))


def test_check_finite_batch_names_the_slice():
    from paper_1203_4587_amd.api import Batch, Slice
    cases = [make_case(32, 16, 6, 3, seed=6), make_case(48, 8, 4, 2, prior="dft", family="periodic", seed=7)]
    dev = [c.device() for c in cases]
    slices = [Slice(dev[0][0], dev[0][1], "tv", 0.1, 0.5, _lib.CS_FLAG_CHECK_FINITE),
              Slice(dev[1][0], dev[1][1], "dft", 0.1, 0.5, _lib.CS_FLAG_CHECK_FINITE)]
    batch = Batch(slices)
    ys = [dev[0][2], dev[1][2].clone()]
    ok = batch.solve(ys, [0.01, 0.01], 6)
    ok = [o.clone() for o in ok]
    t = 0
    ky = int(np.nonzero(cases[1].mask[t])[0][0])
    ys[1][t, 0, ky, 3] = float("nan")
    with pytest.raises(RuntimeError, match="slice 1"):
        batch.solve(ys, [0.01, 0.01], 6)
    ys[1] = dev[1][2]
    again = batch.solve(ys, [0.01, 0.01], 6)
    for a, b in zip(ok, again):
        assert torch.equal(a, b)


def test_eigen_plan_build_allocates_only_through_the_caller():
    """Every device buffer of a CS_FLAG_EIGEN build comes from the caller's
    allocator: the plan's own arrays, and four temporaries of the build (the
    FP64 Gram matrices, eigenvalues with the solver's off-diagonal, the
    solver status, and the eigensolver library's internal workspace, whose
    size the library reports), all four returned before cs_plan_create
    returns.  The plan then solves like a packed plan."""
    from paper_1203_4587_amd.api import Plan
    lib = _lib.load()
    case = make_case(32, 16, 6, 3, seed=8)
    coil, mask, y = case.device()
    events, live = [], {}

    def alloc(nbytes, ctx):
        ptr = torch.cuda.caching_allocator_alloc(int(nbytes), 0)
        live[ptr] = nbytes
        events.append(("a", ptr, nbytes))
        return ptr

    def free(ptr, ctx):
        events.append(("f", ptr, live.pop(ptr)))
        torch.cuda.caching_allocator_delete(ptr)

    a = _lib.CsAllocator(_lib.ALLOC_FN(alloc), _lib.FREE_FN(free), None)
    desc = _lib.CsPlanDesc(32, 16, 6, 3, _lib.CS_PRIOR_TEMPORAL_TV, 0.5, _lib.CS_FLAG_EIGEN)
    h = ctypes.c_void_p()
    st = lib.cs_plan_create(ctypes.byref(desc), ctypes.c_void_p(coil.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
                            0.1, ctypes.byref(a), None, ctypes.byref(h))
    assert st == _lib.CS_OK, lib.cs_last_error()
    freed = [e for e in events if e[0] == "f"]
    assert len(freed) == 4, events
    allocs = [e for e in events if e[0] == "a"]
    nbytes = ctypes.c_size_t()
    assert lib.cs_plan_bytes(h, ctypes.byref(nbytes)) == _lib.CS_OK
    assert sum(live.values()) == nbytes.value
    # the four temporaries are the last four allocations, made after every plan array
    assert {e[1] for e in allocs[-4:]} == {e[1] for e in freed}
    assert lib.cs_plan_destroy(h) == _lib.CS_OK
    assert not live
    eig = Plan(coil, mask, 0.1, prior="tv", flags=_lib.CS_FLAG_EIGEN).solve(y, 0.01, 8)
    xo = O.solve(case.y, case.coil, case.mask, "tv", 0.01, 0.1, 0.5, 8)["x"]
    assert rel_l2(eig.cpu().numpy(), xo) < 1e-4

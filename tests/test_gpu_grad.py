"""GPU parity of the unrolled-ADMM derivative (cs_grad_create, cs_admm_forward_ckpt,
cs_admm_backward and the torch.autograd binding) against the FP64 reference
gradient of the oracle and against FP64 central differences of the oracle's
forward map.  Tolerance 1e-3 (relative l2 for dL/dy, relative for the
scalars).  The 192x192x24, 12-coil, R=8, K=20, checkpoint-every-5 workload
runs at full size with a loss gradient supported on sampled columns, which
the oracle differentiates exactly (columns never interact)."""
import numpy as np
import pytest

import oracle as O
from oracle import gradient as OG
from paper_1203_4587_amd import synthetic as S
from tests.helpers import Case, c64, make_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GTOL = 1e-3
LAM, MU, RHO = 0.02, 0.1, 0.5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rand_c(rng, shape):
    return c64(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def _setup(case, iters, every, flags=0, mu=MU):
    from paper_1203_4587_amd.api import Plan
    from paper_1203_4587_amd.autograd import Unrolled
    coil, mask, y = case.device()
    plan = Plan(coil, mask, mu, prior="tv", mu_ratio=RHO, flags=flags)
    return plan, Unrolled(plan, iters, every), y


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-30)


@pytest.mark.parametrize("every", [1, 3, 7, 50])
def test_forward_ckpt_equals_plain_solve(every):
    from paper_1203_4587_amd import _lib
    case = make_case(48, 32, 8, 3, accel=3, ncenter=2, prior="tv", seed=41)
    for flags in (0, _lib.CS_FLAG_COLUMN_RESIDENT, _lib.CS_FLAG_GRAPH):
        plan, un, y = _setup(case, 12, every, flags)
        x = un.forward_raw(y, LAM, MU)
        assert torch.equal(x, plan.solve(y, LAM, 12)), flags
        un.close()


@pytest.mark.parametrize("shape,iters,every", [((48, 32, 8, 3), 10, 3), ((64, 16, 12, 4), 6, 6),
                                               ((27, 12, 5, 2), 8, 5), ((32, 8, 2, 2), 5, 2),
                                               ((96, 12, 40, 3), 4, 3), ((16, 8, 64, 2), 3, 2)], ids=str)
def test_gradient_matches_oracle_reference(shape, iters, every):
    """dL/dy, dL/dlambda, dL/dmu of L = Re<g, x_K> against the FP64 reverse sweep."""
    nv, nh, nt, nc = shape
    case = make_case(nv, nh, nt, nc, accel=3, ncenter=2, prior="tv", seed=nv * nt + iters, sigma=0.01)
    rng = np.random.default_rng(nv + nt)
    g = _rand_c(rng, case.x_true.shape)
    plan, un, y = _setup(case, iters, every)
    un.forward_raw(y, LAM, MU)
    gy, gs = un.backward_raw(torch.from_numpy(g.astype(np.complex64)).cuda())
    ref = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, MU, RHO, iters, g)
    ey = rel_l2(gy.cpu().numpy(), ref["y"])
    el, em = _rel(float(gs[0]), ref["lam"]), _rel(float(gs[1]), ref["mu"])
    print(shape, iters, every, "dy", ey, "dlam", el, "dmu", em)
    assert ey < GTOL and el < GTOL and em < GTOL
    # a second backward of the same forward is identical
    gy2, gs2 = un.backward_raw(torch.from_numpy(g.astype(np.complex64)).cuda())
    assert torch.equal(gy, gy2) and torch.equal(gs, gs2)


def test_checkpoint_schedule_does_not_change_gradients():
    """Every checkpoint interval runs the same kernels in the same order: the
    gradients for ckpt_every = 1, 4 and K (the forward keeps the whole tape,
    nothing is recomputed) are bit-identical."""
    case = make_case(48, 32, 8, 3, accel=3, ncenter=2, prior="tv", seed=77, sigma=0.01)
    rng = np.random.default_rng(5)
    g = torch.from_numpy(_rand_c(rng, case.x_true.shape).astype(np.complex64)).cuda()
    out = []
    for every in (1, 4, 9):
        plan, un, y = _setup(case, 9, every)
        un.forward_raw(y, LAM, MU)
        out.append(un.backward_raw(g))
        un.close()
    for gy, gs in out[1:]:
        assert torch.equal(gy, out[0][0]) and torch.equal(gs, out[0][1])


def test_gradient_matches_fp64_finite_differences():
    """The GPU gradient against central differences of the oracle's FP64
    forward map (y along a random sampled direction, lambda, mu)."""
    case = make_case(32, 16, 6, 3, accel=3, ncenter=2, prior="tv", seed=8, sigma=0.01)
    K = 8
    rng = np.random.default_rng(9)
    g = _rand_c(rng, case.x_true.shape)
    plan, un, y = _setup(case, K, 3)
    un.forward_raw(y, LAM, MU)
    gy, gs = un.backward_raw(torch.from_numpy(g.astype(np.complex64)).cuda())
    fac = O.BlockFactor(case.coil, case.mask)
    L = lambda yy=case.y, lam=LAM, mu=MU: OG.unrolled_tv_loss(yy, case.coil, case.mask, lam, mu, RHO, K, g, fac=fac)
    h = 1e-6
    dy = (rng.standard_normal(case.y.shape) + 1j * rng.standard_normal(case.y.shape)) * case.mask[:, None, :, None]
    fd_y = (L(yy=case.y + h * dy) - L(yy=case.y - h * dy)) / (2 * h)
    an_y = float(np.real(np.vdot(gy.cpu().numpy().astype(np.complex128), dy)))
    fd_l = (L(lam=LAM + h) - L(lam=LAM - h)) / (2 * h)
    fd_m = (L(mu=MU + h) - L(mu=MU - h)) / (2 * h)
    print("fd y", fd_y, an_y, "lam", fd_l, float(gs[0]), "mu", fd_m, float(gs[1]))
    assert _rel(an_y, fd_y) < GTOL
    assert _rel(float(gs[0]), fd_l) < GTOL
    assert _rel(float(gs[1]), fd_m) < GTOL


def test_autograd_function_and_losses():
    """torch.autograd drives the same kernels: y.grad, lam.grad, mu.grad of
    Re<g, x> equal backward_raw(g); the squared-error loss passes its own
    gradient 2 (x - x_true) through."""
    case = make_case(48, 16, 8, 3, accel=3, ncenter=2, prior="tv", seed=13, sigma=0.01)
    rng = np.random.default_rng(14)
    g = torch.from_numpy(_rand_c(rng, case.x_true.shape).astype(np.complex64)).cuda()
    plan, un, y = _setup(case, 9, 4)
    yv = y.clone().requires_grad_(True)
    lam = torch.tensor(LAM, requires_grad=True)
    mu = torch.tensor(MU, requires_grad=True)
    x = un(yv, lam, mu)
    torch.real(torch.sum(torch.conj(g) * x)).backward()
    un.forward_raw(y, LAM, MU)
    gy, gs = un.backward_raw(g)
    assert torch.equal(yv.grad, gy)
    assert lam.grad.item() == float(gs[0]) and mu.grad.item() == float(gs[1])
    xt = torch.from_numpy(case.x_true.astype(np.complex64)).cuda()
    yv.grad = None
    x = un(yv, LAM, MU)
    loss = torch.sum(torch.abs(x - xt) ** 2)
    loss.backward()
    un.forward_raw(y, LAM, MU)
    gy2, _ = un.backward_raw(2 * (x.detach() - xt))
    assert torch.allclose(yv.grad, gy2, rtol=1e-5, atol=1e-6 * float(gy2.abs().max()))
    # a second forward before the first backward is refused
    a = un(yv, LAM, MU)
    b = un(yv, LAM, MU)
    with pytest.raises(RuntimeError, match="another forward"):
        torch.real(a.sum()).backward()
    del b


def test_zero_iterations_and_errors():
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    from paper_1203_4587_amd.autograd import Unrolled
    case = make_case(32, 16, 6, 2, prior="tv", seed=2)
    plan, un, y = _setup(case, 0, 5)
    x = un.forward_raw(y, LAM, MU)
    assert torch.equal(x, plan.solve(y, LAM, 0))
    rng = np.random.default_rng(3)
    g = torch.from_numpy(_rand_c(rng, case.x_true.shape).astype(np.complex64)).cuda()
    gy, gs = un.backward_raw(g)
    assert torch.allclose(gy, plan.apply_A(g), rtol=1e-6, atol=1e-6)
    assert float(gs[0]) == 0.0 and float(gs[1]) == 0.0
    fresh = Unrolled(plan, 4, 2)
    with pytest.raises(_lib.CsmriError, match="preceding"):
        fresh.backward_raw(g)
    coil, mask, _ = case.device()
    frame = Plan(coil, mask, MU, prior="frame")
    h = __import__("ctypes").c_void_p()
    assert _lib.load().cs_grad_create(frame.handle, 4, 2, __import__("ctypes").byref(h)) == _lib.CS_EUNSUPPORTED


def test_full_size_192x192x24_12c_k20_ckpt5_sampled_columns():
    """The 192x192x24, 12-coil, R=8 workload, K = 20 unrolled iterations with a
    checkpoint every 5, in full; the loss gradient lives on two columns so
    the oracle's reverse sweep covers it exactly."""
    pr = S.CONFIGS["tv192_unrolled"]()
    case = Case(pr)
    nt, nv, nh = pr.x_true.shape
    cols = np.array([5, 131])
    rng = np.random.default_rng(1005)
    gcols = _rand_c(rng, (nt, nv, cols.size))
    g = np.zeros((nt, nv, nh), dtype=np.complex128)
    g[:, :, cols] = gcols
    plan, un, y = _setup(case, pr.iters, 5, mu=pr.mu)
    un.forward_raw(y, pr.lam, pr.mu)
    gy, gs = un.backward_raw(torch.from_numpy(g.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    ref = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, pr.lam, pr.mu, pr.rho, pr.iters, gcols, cols=cols)
    ey = rel_l2(gy.cpu().numpy(), ref["y"])
    el, em = _rel(float(gs[0]), ref["lam"]), _rel(float(gs[1]), ref["mu"])
    print("192x192x24 K=20: dy", ey, "dlam", el, "dmu", em)
    assert ey < GTOL and el < GTOL and em < GTOL


@pytest.mark.parametrize("prior", ["tv", "dft"])
def test_mu_other_than_the_plans_refactors(prior):
    """A forward with a mu different from the plan's refactors the plan (as
    cs_admm_solve does) and gives the image and gradients of a plan built
    with that mu; with CS_FLAG_NO_REFACTOR the call is refused."""
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    from paper_1203_4587_amd.autograd import Unrolled
    fam = "cardiac" if prior == "tv" else "periodic"
    case = make_case(48, 16, 8, 3, accel=3, ncenter=2, prior=prior, family=fam, seed=91, sigma=0.01)
    coil, mask, y = case.device()
    rng = np.random.default_rng(92)
    g = torch.from_numpy(_rand_c(rng, case.x_true.shape).astype(np.complex64)).cuda()
    mu2 = 0.25
    a = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO)
    ua = Unrolled(a, 6, 3)
    xa = ua.forward_raw(y, LAM, mu2)
    gya, gsa = ua.backward_raw(g)
    b = Plan(coil, mask, mu2, prior=prior, mu_ratio=RHO)
    ub = Unrolled(b, 6, 3)
    xb = ub.forward_raw(y, LAM, mu2)
    gyb, gsb = ub.backward_raw(g)
    assert torch.equal(xa, xb) and torch.equal(gya, gyb) and torch.equal(gsa, gsb)
    c = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=_lib.CS_FLAG_NO_REFACTOR)
    uc = Unrolled(c, 6, 3)
    with pytest.raises(_lib.CsmriError, match="mu"):
        uc.forward_raw(y, LAM, mu2)

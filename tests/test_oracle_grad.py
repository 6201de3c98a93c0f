"""Pins of the FP64 reference gradient of unrolled Algorithm 2 (oracle/gradient.py).

The reverse sweep is checked against things that do not share its
derivation: central finite differences of the oracle's own forward map in
FP64 (in y along random complex directions, in lambda and in mu), the exact
adjoint identity of the map at lambda = 0 (where it is linear in y), the
closed form at K = 0, finite differences of the soft threshold alone, and
the complex-gradient convention of torch.autograd that the GPU binding must
follow.  A dropped term (e.g. the derivative of (mu I + H'H)^{-1} in mu), a
wrong sign or a transposed operator in any line fails at least one of these."""
import numpy as np
import pytest

import oracle as O
from oracle import gradient as OG
from tests.helpers import make_case

LAM, MU, RHO = 0.05, 0.1, 0.5


def _rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _tiny(seed=3, nv=8, nh=6, nt=5, nc=2):
    return make_case(nv, nh, nt, nc, accel=2, ncenter=2, prior="tv", seed=seed, sigma=0.02)


def test_torch_complex_gradient_convention():
    """torch.autograd's gradient of a real loss w.r.t. a complex tensor is
    dL/dRe z + i dL/dIm z: |z|^2 gives 2z and Re<g, z> gives g."""
    torch = pytest.importorskip("torch")
    z = torch.randn(7, dtype=torch.complex128, requires_grad=True)
    (z.abs() ** 2).sum().backward()
    assert torch.allclose(z.grad, 2 * z.detach())
    g = torch.randn(7, dtype=torch.complex128)
    z.grad = None
    torch.real(torch.sum(torch.conj(g) * z)).backward()
    assert torch.allclose(z.grad, g)


def test_soft_vjp_matches_finite_differences():
    rng = np.random.default_rng(0)
    a = _rand_c(rng, 200)
    tau = 0.7
    a = a[np.abs(np.abs(a) - tau) > 1e-3]          # away from the kink
    gv = _rand_c(rng, a.shape)
    da = _rand_c(rng, a.shape)
    h = 1e-6
    L = lambda aa, tt: float(np.real(np.vdot(gv, O.soft(aa, tt))))
    fd_a = (L(a + h * da, tau) - L(a - h * da, tau)) / (2 * h)
    fd_t = (L(a, tau + h) - L(a, tau - h)) / (2 * h)
    ga, gt = OG.soft_vjp(a, tau, gv)
    assert abs(float(np.real(np.vdot(ga, da))) - fd_a) < 1e-8 * max(1.0, abs(fd_a))
    assert abs(gt - fd_t) < 1e-8 * max(1.0, abs(fd_t))
    # below the threshold nothing passes
    small = 0.5 * tau * np.exp(1j * rng.uniform(0, 2 * np.pi, 10))
    ga0, gt0 = OG.soft_vjp(small, tau, _rand_c(rng, 10))
    assert np.all(ga0 == 0) and gt0 == 0.0


def test_zero_iterations_gradient_is_forward_operator():
    """K = 0: x_K = H'y, so dL/dy = A(g) and nothing depends on lambda or mu."""
    case = _tiny()
    rng = np.random.default_rng(1)
    g = _rand_c(rng, case.x_true.shape)
    res = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, MU, RHO, 0, g)
    assert np.allclose(res["y"], O.forward(g, case.coil, case.mask), atol=1e-14)
    assert res["lam"] == 0.0 and res["mu"] == 0.0


def test_linear_case_adjoint_identity():
    """lambda = 0 makes every step linear in y, so L(y) = Re<g, x_K(y)> equals
    Re<dL/dy, y> exactly (to rounding), with no finite-difference step."""
    case = _tiny(seed=5)
    rng = np.random.default_rng(2)
    g = _rand_c(rng, case.x_true.shape)
    for K in (1, 4, 9):
        res = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, 0.0, MU, RHO, K, g)
        L = OG.unrolled_tv_loss(case.y, case.coil, case.mask, 0.0, MU, RHO, K, g)
        lin = float(np.real(np.vdot(res["y"], case.y)))
        assert abs(L - lin) < 1e-12 * max(1.0, abs(L)), (K, L, lin)
        # unsampled rows of y never reach the result
        for t in range(case.mask.shape[0]):
            assert np.all(res["y"][t][:, case.mask[t] == 0, :] == 0)


@pytest.mark.parametrize("K", [1, 3, 8])
def test_unrolled_gradient_matches_central_differences(K):
    case = _tiny(seed=7 + K)
    rng = np.random.default_rng(10 + K)
    g = _rand_c(rng, case.x_true.shape)
    res = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, MU, RHO, K, g)
    fac = O.BlockFactor(case.coil, case.mask)
    L = lambda y=case.y, lam=LAM, mu=MU: OG.unrolled_tv_loss(y, case.coil, case.mask, lam, mu, RHO, K, g, fac=fac)
    h = 1e-6
    # y along a random complex direction on the sampled rows
    dy = _rand_c(rng, case.y.shape) * case.mask[:, None, :, None]
    fd_y = (L(y=case.y + h * dy) - L(y=case.y - h * dy)) / (2 * h)
    an_y = float(np.real(np.vdot(res["y"], dy)))
    assert abs(fd_y - an_y) < 1e-6 * max(abs(an_y), 1e-3), (fd_y, an_y)
    fd_l = (L(lam=LAM + h) - L(lam=LAM - h)) / (2 * h)
    assert abs(fd_l - res["lam"]) < 1e-6 * max(abs(res["lam"]), 1e-3), (fd_l, res["lam"])
    fd_m = (L(mu=MU + h) - L(mu=MU - h)) / (2 * h)
    assert abs(fd_m - res["mu"]) < 1e-6 * max(abs(res["mu"]), 1e-3), (fd_m, res["mu"])
    # the thresholds were active: lambda really matters here
    assert abs(res["lam"]) > 1e-3


def test_squared_error_loss_gradient():
    """L = ||x_K - x_true||^2 has dL/dx_K = 2 (x_K - x_true); checked by
    central differences of the loss itself in y and mu."""
    case = _tiny(seed=21)
    K = 5
    fac = O.BlockFactor(case.coil, case.mask)

    def loss(y, mu):
        Hy = O.adjoint_columns(y, case.coil, case.mask, np.arange(case.coil.shape[2]))
        xK, _ = OG.unrolled_tv_forward(Hy, fac, LAM, mu, RHO, K)
        return float(np.sum(np.abs(xK - case.x_true) ** 2)), xK

    _, xK = loss(case.y, MU)
    res = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, MU, RHO, K, 2 * (xK - case.x_true), fac=fac)
    rng = np.random.default_rng(4)
    dy = _rand_c(rng, case.y.shape) * case.mask[:, None, :, None]
    h = 1e-6
    fd_y = (loss(case.y + h * dy, MU)[0] - loss(case.y - h * dy, MU)[0]) / (2 * h)
    an_y = float(np.real(np.vdot(res["y"], dy)))
    assert abs(fd_y - an_y) < 1e-6 * max(abs(an_y), 1e-3)
    fd_m = (loss(case.y, MU + h)[0] - loss(case.y, MU - h)[0]) / (2 * h)
    assert abs(fd_m - res["mu"]) < 1e-6 * max(abs(res["mu"]), 1e-3)


def test_column_restriction_equals_full_sweep():
    """With g supported on a few columns, the column-restricted sweep gives the
    full sweep's dL/dy, dL/dlambda, dL/dmu (columns never interact)."""
    case = _tiny(seed=31, nh=8)
    rng = np.random.default_rng(6)
    cols = np.array([1, 6])
    g = np.zeros(case.x_true.shape, dtype=np.complex128)
    g[:, :, cols] = _rand_c(rng, (g.shape[0], g.shape[1], cols.size))
    full = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, MU, RHO, 4, g)
    part = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, MU, RHO, 4, g[:, :, cols], cols=cols)
    assert np.allclose(part["y"], full["y"], rtol=1e-12, atol=1e-13)
    assert abs(part["lam"] - full["lam"]) < 1e-12 * max(1.0, abs(full["lam"]))
    assert abs(part["mu"] - full["mu"]) < 1e-12 * max(1.0, abs(full["mu"]))


# ---------------------------------------------------------------- Algorithm 1 (temporal DFT)

def _tiny_dft(seed=3, nv=8, nh=6, nt=6, nc=2):
    return make_case(nv, nh, nt, nc, accel=2, ncenter=2, prior="dft", family="periodic", seed=seed, sigma=0.02)


def test_dft_unrolled_forward_equals_algorithm_1():
    """The differentiated forward map is Algorithm 1 as the solver oracle runs
    it (which keeps the general tight-frame w-update)."""
    case = _tiny_dft()
    fac = O.BlockFactor(case.coil, case.mask)
    Hy = O.adjoint(case.y, case.coil, case.mask)
    for K in (0, 1, 6):
        xK, _ = OG.unrolled_dft_forward(Hy, fac, LAM, MU, K)
        ref = O.admm_synthesis(Hy, fac, LAM, MU, K)["x"]
        assert np.allclose(xK, ref, rtol=1e-12, atol=1e-13), K


def test_dft_zero_iterations_gradient_is_forward_operator():
    case = _tiny_dft(seed=2)
    rng = np.random.default_rng(1)
    g = _rand_c(rng, case.x_true.shape)
    res = OG.unrolled_dft_grad_y(case.y, case.coil, case.mask, LAM, MU, 0, g)
    assert np.allclose(res["y"], O.forward(g, case.coil, case.mask), atol=1e-14)
    assert res["lam"] == 0.0 and res["mu"] == 0.0


def test_dft_linear_case_adjoint_identity():
    """lambda = 0: soft(a, 0) = a, so the unrolled map is linear in y and
    L(y) = Re<dL/dy, y> holds exactly."""
    case = _tiny_dft(seed=5)
    rng = np.random.default_rng(2)
    g = _rand_c(rng, case.x_true.shape)
    for K in (1, 4, 9):
        res = OG.unrolled_dft_grad_y(case.y, case.coil, case.mask, 0.0, MU, K, g)
        L = OG.unrolled_dft_loss(case.y, case.coil, case.mask, 0.0, MU, K, g)
        lin = float(np.real(np.vdot(res["y"], case.y)))
        assert abs(L - lin) < 1e-12 * max(1.0, abs(L)), (K, L, lin)


@pytest.mark.parametrize("K", [1, 3, 8])
def test_dft_unrolled_gradient_matches_central_differences(K):
    case = _tiny_dft(seed=7 + K)
    rng = np.random.default_rng(10 + K)
    g = _rand_c(rng, case.x_true.shape)
    res = OG.unrolled_dft_grad_y(case.y, case.coil, case.mask, LAM, MU, K, g)
    fac = O.BlockFactor(case.coil, case.mask)
    L = lambda y=case.y, lam=LAM, mu=MU: OG.unrolled_dft_loss(y, case.coil, case.mask, lam, mu, K, g, fac=fac)
    h = 1e-6
    dy = _rand_c(rng, case.y.shape) * case.mask[:, None, :, None]
    fd_y = (L(y=case.y + h * dy) - L(y=case.y - h * dy)) / (2 * h)
    an_y = float(np.real(np.vdot(res["y"], dy)))
    assert abs(fd_y - an_y) < 1e-6 * max(abs(an_y), 1e-3), (fd_y, an_y)
    fd_l = (L(lam=LAM + h) - L(lam=LAM - h)) / (2 * h)
    assert abs(fd_l - res["lam"]) < 1e-6 * max(abs(res["lam"]), 1e-3), (fd_l, res["lam"])
    fd_m = (L(mu=MU + h) - L(mu=MU - h)) / (2 * h)
    assert abs(fd_m - res["mu"]) < 1e-6 * max(abs(res["mu"]), 1e-3), (fd_m, res["mu"])
    assert abs(res["lam"]) > 1e-3


def test_dft_column_restriction_equals_full_sweep():
    case = _tiny_dft(seed=31, nh=8)
    rng = np.random.default_rng(6)
    cols = np.array([0, 5])
    g = np.zeros(case.x_true.shape, dtype=np.complex128)
    g[:, :, cols] = _rand_c(rng, (g.shape[0], g.shape[1], cols.size))
    full = OG.unrolled_dft_grad_y(case.y, case.coil, case.mask, LAM, MU, 4, g)
    part = OG.unrolled_dft_grad_y(case.y, case.coil, case.mask, LAM, MU, 4, g[:, :, cols], cols=cols)
    assert np.allclose(part["y"], full["y"], rtol=1e-12, atol=1e-13)
    assert abs(part["lam"] - full["lam"]) < 1e-12 * max(1.0, abs(full["lam"]))
    assert abs(part["mu"] - full["mu"]) < 1e-12 * max(1.0, abs(full["mu"]))


@pytest.mark.parametrize("prior", ["tv", "dft"])
@pytest.mark.parametrize("plant", ["jacobian_sign", "jacobian_conjugate", "tau_sign"])
def test_planted_mistakes_fail_the_pins(prior, plant, monkeypatch):
    """A mistake planted in the oracle's reverse sweep (here in the soft
    threshold's transposed Jacobian, shared by both sweeps) is caught by the
    central-difference pins: the planted sweep disagrees with the differences
    of the (unchanged) forward map."""
    good = OG.soft_vjp

    def planted(a, tau, gv):
        ga, gt = good(a, tau, gv)
        if plant == "jacobian_sign":
            return -ga, gt
        if plant == "jacobian_conjugate":
            return np.conj(ga), gt
        return ga, -gt

    monkeypatch.setattr(OG, "soft_vjp", planted)
    K = 3
    case = _tiny(seed=12) if prior == "tv" else _tiny_dft(seed=12)
    rng = np.random.default_rng(40)
    g = _rand_c(rng, case.x_true.shape)
    fac = O.BlockFactor(case.coil, case.mask)
    if prior == "tv":
        res = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, MU, RHO, K, g, fac=fac)
        L = lambda y=case.y, lam=LAM: OG.unrolled_tv_loss(y, case.coil, case.mask, lam, MU, RHO, K, g, fac=fac)
    else:
        res = OG.unrolled_dft_grad_y(case.y, case.coil, case.mask, LAM, MU, K, g, fac=fac)
        L = lambda y=case.y, lam=LAM: OG.unrolled_dft_loss(y, case.coil, case.mask, lam, MU, K, g, fac=fac)
    h = 1e-6
    dy = _rand_c(rng, case.y.shape) * case.mask[:, None, :, None]
    fd_y = (L(y=case.y + h * dy) - L(y=case.y - h * dy)) / (2 * h)
    an_y = float(np.real(np.vdot(res["y"], dy)))
    fd_l = (L(lam=LAM + h) - L(lam=LAM - h)) / (2 * h)
    y_ok = abs(fd_y - an_y) < 1e-6 * max(abs(an_y), 1e-3)
    l_ok = abs(fd_l - res["lam"]) < 1e-6 * max(abs(res["lam"]), 1e-3)
    assert not (y_ok and l_ok), (plant, fd_y, an_y, fd_l, res["lam"])

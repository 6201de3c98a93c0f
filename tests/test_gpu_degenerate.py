"""GPU parity in the degenerate cases the method admits, against the FP64
oracle after a fixed iteration count (relative l2 1e-4): lambda = 0 (every
shrinkage is the identity: the least-squares iteration), full sampling
(R = 1: every block of H'H is the identity for sum-of-squares maps), a single
coil, a lambda so large that every coefficient is thresholded away, and zero
data (the iterates stay exactly zero)."""
import numpy as np
import pytest

import oracle as O
from tests.helpers import c64, make_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-4
MU, RHO = 0.1, 0.5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(case, prior, lam, iters):
    from paper_1203_4587_amd.api import Plan
    coil, mask, y = case.device()
    plan = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO)
    return plan.solve(y, lam, iters).cpu().numpy()


def _case(prior, **kw):
    fam = "cardiac" if prior == "tv" else "periodic"
    args = dict(nv=48, nh=16, nt=8, nc=3, accel=3, ncenter=2, seed=61)
    args.update(kw)
    return make_case(args["nv"], args["nh"], args["nt"], args["nc"], accel=args["accel"], ncenter=args["ncenter"],
                     prior=prior, family=fam, seed=args["seed"], sigma=0.01)


@pytest.mark.parametrize("prior", ["tv", "dft"])
@pytest.mark.parametrize("what", ["lambda0", "full_sampling", "single_coil", "huge_lambda"])
def test_degenerate_cases_match_oracle(prior, what):
    lam, iters = 0.02, 15
    if what == "lambda0":
        case, lam = _case(prior), 0.0
    elif what == "full_sampling":
        # every phase-encode row of every frame (the variable-density draw
        # never picks the Nyquist row, so the mask is set here)
        case = _case(prior)
        case.mask = np.ones_like(case.mask)
        case.y = c64(O.forward(case.x_true, case.coil, case.mask))
    elif what == "single_coil":
        case = _case(prior, nc=1)
    else:
        case, lam = _case(prior), 1e4
    x = _solve(case, prior, lam, iters)
    ref = O.solve(case.y, case.coil, case.mask, prior, lam, MU, RHO, iters)["x"]
    err = rel_l2(x, ref)
    print(prior, what, "rel_l2", err)
    assert err < TOL


@pytest.mark.parametrize("prior", ["tv", "dft", "frame"])
def test_zero_data_gives_zero_iterates(prior):
    from paper_1203_4587_amd.api import Plan
    case = _case("dft" if prior == "frame" else prior)
    coil, mask, y = case.device()
    plan = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO)
    st = plan.new_state()
    x = plan.solve(torch.zeros_like(y), 0.02, 10, state=st)
    assert not x.any()
    for n in ("s0", "s1", "s2"):
        assert not getattr(st, n).any(), n

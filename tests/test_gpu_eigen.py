"""GPU parity of the eigen-form factor (CS_FLAG_EIGEN: G = U diag(e) U' per
block, Sec. IV-C eq. eigen_mu) against the FP64 oracle, which applies the
block inverse in that same form, through the C ABI.  Tolerances as for the
packed inverse: relative l2 <= 1e-4 for solves, 1e-3 for gradients."""
import numpy as np
import pytest

import oracle as O
import oracle.gradient as OG
from tests.helpers import c64, make_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL, GTOL = 1e-4, 1e-3
LAM, MU, RHO = 0.02, 0.1, 0.5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _flag():
    from paper_1203_4587_amd import _lib
    return _lib.CS_FLAG_EIGEN


def _case(shape, prior, seed):
    nv, nh, nt, nc = shape
    fam = "cardiac" if prior == "tv" else "periodic"
    kind = "tv" if prior == "tv" else "dft"
    return make_case(nv, nh, nt, nc, accel=3, ncenter=2, prior=kind, family=fam, seed=seed, sigma=0.01)


@pytest.mark.parametrize("shape,prior,iters", [
    ((64, 16, 8, 3), "tv", 25),
    ((48, 12, 6, 2), "dft", 25),
    ((27, 12, 4, 2), "tv", 20),       # odd nv, part of the wave idle
    ((192, 4, 3, 2), "dft", 10),      # three indices per lane
    ((384, 3, 2, 2), "tv", 8),        # six indices per lane
    ((512, 2, 2, 2), "dft", 6),       # maximum nv
    ((16, 8, 6, 2), "frame", 15),
    ((2, 4, 3, 1), "tv", 10),         # smallest block
], ids=lambda v: str(v))
def test_eigen_solves_match_oracle(shape, prior, iters):
    from paper_1203_4587_amd.api import Plan
    case = _case(shape, prior, seed=sum(shape) + iters)
    coil, mask, y = case.device()
    plan = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=_flag())
    x = plan.solve(y, LAM, iters)
    ref = O.solve(case.y, case.coil, case.mask, prior, LAM, MU, RHO, iters)
    err = rel_l2(x.cpu().numpy(), ref["x"])
    print(shape, prior, "rel_l2", err)
    assert err < TOL


@pytest.mark.parametrize("prior", ["tv", "dft"])
def test_any_mu_without_refactoring(prior):
    """One eigen plan serves every mu: a solve at a mu other than the plan's
    runs under CS_FLAG_NO_REFACTOR (a packed-inverse plan refuses it), matches
    the oracle at that mu and agrees with a packed plan built for it."""
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    case = _case((64, 12, 6, 3), prior, seed=5)
    coil, mask, y = case.device()
    eig = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=_flag() | _lib.CS_FLAG_NO_REFACTOR)
    packed = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=_lib.CS_FLAG_NO_REFACTOR)
    for mu in (0.35, 0.03, MU):
        x = eig.solve(y, LAM, 15, mu=mu)
        ref = O.solve(case.y, case.coil, case.mask, prior, LAM, mu, RHO, 15)
        assert rel_l2(x.cpu().numpy(), ref["x"]) < TOL, mu
        if mu != MU:
            with pytest.raises(_lib.CsmriError, match="mu"):
                packed.solve(y, LAM, 15, mu=mu)
        fresh = Plan(coil, mask, mu, prior=prior, mu_ratio=RHO)
        xp = fresh.solve(y, LAM, 15)
        assert rel_l2(x.cpu().numpy(), xp.cpu().numpy()) < TOL, mu


@pytest.mark.parametrize("shape", [(64, 16, 4, 3), (27, 6, 2, 3), (256, 4, 2, 8), (2, 4, 2, 1)],
                         ids=lambda s: "x".join(map(str, s)))
def test_eigen_block_inverse_matches_oracle(shape):
    from paper_1203_4587_amd.api import Plan, to_device
    nv, nh, nt, nc = shape
    case = make_case(nv, nh, nt, nc, accel=3, ncenter=2, seed=nv + nh)
    coil, mask, _ = case.device()
    mu = 0.07
    plan = Plan(coil, mask, mu, prior="tv", mu_ratio=RHO, flags=_flag())
    fac = O.BlockFactor(case.coil, case.mask)
    rng = np.random.default_rng(4)
    b = c64(rng.standard_normal((nt, nv, nh)) + 1j * rng.standard_normal((nt, nv, nh)))
    x_gpu = plan.block_inverse(to_device(b)).cpu().numpy()
    assert rel_l2(x_gpu, fac.solve(b, mu)) < 2e-6
    # residual of one block system, from the oracle's Gram block
    t, i = nt - 1, nh // 2
    G = O.gram_block(case.coil[:, :, i], case.mask[t])
    r = (mu * np.eye(nv) + G) @ x_gpu[t, :, i] - b[t, :, i]
    assert np.linalg.norm(r) <= 1e-5 * np.linalg.norm(b[t, :, i])


def test_flag_is_fixed_at_creation_and_forms_are_ignored():
    """cs_plan_set_flags neither adds nor removes CS_FLAG_EIGEN; the
    execution-form flags (column-resident, wave, group) leave an eigen plan's
    result bit-identical."""
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    case = _case((32, 8, 6, 2), "tv", seed=11)
    coil, mask, y = case.device()
    plan = Plan(coil, mask, MU, prior="tv", mu_ratio=RHO, flags=_flag())
    nt, nv, nh = plan.image_shape
    assert plan.nbytes >= 2 * nt * nh * nv * nv * 8 + nt * nh * nv * 4   # U twice and e
    ref = plan.solve(y, LAM, 10)
    for f in (_lib.CS_FLAG_COLUMN_RESIDENT, _lib.CS_FLAG_XU_WAVE, _lib.CS_FLAG_XU_GROUP | _lib.CS_FLAG_GRAPH, 0):
        plan.flags = f
        assert plan.flags & _flag()
        assert torch.equal(plan.solve(y, LAM, 10), ref), f
    # graph replays of the eigen x-update, with eager work in between
    plan.flags = _lib.CS_FLAG_GRAPH
    for rep in range(3):
        assert torch.equal(plan.solve(y, LAM, 10), ref), rep
        plan.apply_AH(y)
        torch.cuda.synchronize()
    packed = Plan(coil, mask, MU, prior="tv", mu_ratio=RHO)
    packed.flags = _flag()
    assert not packed.flags & _flag()


@pytest.mark.parametrize("prior", ["tv", "dft"])
def test_eigen_gradients_match_oracle(prior):
    """Reverse mode of an unrolled solve on an eigen plan, at a mu other than
    the plan's, against the FP64 reverse sweeps."""
    from paper_1203_4587_amd.api import Plan
    from paper_1203_4587_amd.autograd import Unrolled
    case = _case((48, 16, 8, 3), prior, seed=23)
    coil, mask, y = case.device()
    rng = np.random.default_rng(24)
    g = c64(rng.standard_normal(case.x_true.shape) + 1j * rng.standard_normal(case.x_true.shape))
    mu = 0.15
    plan = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=_flag())
    un = Unrolled(plan, 8, 3)
    un.forward_raw(y, LAM, mu)
    gy, gs = un.backward_raw(torch.from_numpy(g.astype(np.complex64)).cuda())
    if prior == "tv":
        ref = OG.unrolled_tv_grad_y(case.y, case.coil, case.mask, LAM, mu, RHO, 8, g)
    else:
        ref = OG.unrolled_dft_grad_y(case.y, case.coil, case.mask, LAM, mu, 8, g)
    ey = rel_l2(gy.cpu().numpy(), ref["y"])
    el = abs(float(gs[0]) - ref["lam"]) / abs(ref["lam"])
    em = abs(float(gs[1]) - ref["mu"]) / abs(ref["mu"])
    print(prior, "dy", ey, "dlam", el, "dmu", em)
    assert ey < GTOL and el < GTOL and em < GTOL


def test_eigen_batch_slice():
    """An eigen-form slice inside a batch gives the result of its own plan."""
    from paper_1203_4587_amd.api import Batch, Plan, Slice
    cases = [_case((32, 8, 6, 2), "tv", seed=31), _case((48, 6, 4, 2), "dft", seed=32)]
    slices, ys, refs = [], [], []
    for c, prior in zip(cases, ("tv", "dft")):
        coil, mask, y = c.device()
        slices.append(Slice(coil, mask, prior, MU, RHO, flags=_flag()))
        ys.append(y)
        refs.append(Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=_flag()).solve(y, LAM, 12))
    xs = Batch(slices).solve(ys, [LAM, LAM], 12)
    for x, r in zip(xs, refs):
        assert torch.equal(x, r)


@pytest.mark.parametrize("prior", ["tv", "dft"])
@pytest.mark.parametrize("what", ["empty_frame", "full_sampling"])
def test_eigen_degenerate_blocks(prior, what):
    """Blocks whose eigendecomposition is degenerate: a frame with no sampled
    line (G = 0: every e = 0, x = b / mu) and full sampling (G = I for
    sum-of-squares maps: one eigenvalue of multiplicity nv, U any orthonormal
    basis)."""
    from paper_1203_4587_amd.api import Plan
    case = _case((48, 16, 8, 3), prior, seed=61)
    if what == "empty_frame":
        case.mask[3] = 0
    else:
        case.mask = np.ones_like(case.mask)
    case.y = c64(O.forward(case.x_true, case.coil, case.mask))
    coil, mask, y = case.device()
    plan = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=_flag())
    x = plan.solve(y, LAM, 15).cpu().numpy()
    ref = O.solve(case.y, case.coil, case.mask, prior, LAM, MU, RHO, 15)["x"]
    err = rel_l2(x, ref)
    print(prior, what, "rel_l2", err)
    assert err < TOL


def test_eigen_full_size_tv_256x256x32_8c_sampled_columns():
    """The 256x256x32, 8-coil, R=8 temporal-TV workload at full size on an
    eigen-form plan, at the benchmark's iteration count; the oracle recomputes
    five columns exactly (temporal priors never couple columns)."""
    from paper_1203_4587_amd import synthetic as S
    from paper_1203_4587_amd.api import Plan
    from tests.helpers import Case
    case = Case(S.CONFIGS["tv256"]())
    p = case.p
    coil, mask, y = case.device()
    plan = Plan(coil, mask, p.mu, prior="tv", mu_ratio=p.rho, flags=_flag())
    x = plan.solve(y, p.lam, p.iters).cpu().numpy()
    nh = p.x_true.shape[2]
    cols = np.array(sorted({0, 1, nh // 3, nh // 2 + 1, nh - 1}))
    ref = O.solve(case.y, case.coil, case.mask, "tv", p.lam, p.mu, p.rho, p.iters, cols=cols)
    err = rel_l2(x[:, :, cols], ref["x"])
    print("tv256 eigen sampled rel_l2", err)
    assert err < TOL

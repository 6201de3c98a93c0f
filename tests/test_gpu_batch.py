"""GPU parity of batched solves (cs_batch_create / cs_batch_solve), the
x-update form flags and the autotuner, through the C ABI.

A batch runs each slice's own kernels, so every slice must equal a plain
cs_admm_solve of that slice bit for bit, and the oracle of that slice within
relative l2 1e-4.  The 24-slice uneven workload (128x96x16 with 8 coils at
R=4 up to 256x256x40 with 16 coils at R=10, both priors) is checked at full
size on sampled columns, which the oracle computes exactly because temporal
priors never couple columns."""
import numpy as np
import pytest

import oracle as O
from paper_1203_4587_amd import synthetic as S
from tests.helpers import Case, make_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# uneven shapes, coil counts and priors; odd nv (no column-resident form),
# two frames, one frame
SMALL = [((48, 32, 8, 3), "tv"), ((64, 24, 12, 4), "dft"), ((27, 16, 5, 2), "tv"),
         ((96, 12, 6, 5), "dft"), ((32, 8, 2, 2), "tv"), ((16, 8, 1, 2), "dft")]
LAMS = [0.02, 0.01, 0.03, 0.015, 0.02, 0.05]
MU, RHO = 0.1, 0.5


def _small_cases():
    out = []
    for k, ((nv, nh, nt, nc), prior) in enumerate(SMALL):
        fam = "cardiac" if prior == "tv" else "periodic"
        out.append(make_case(nv, nh, nt, nc, accel=3, ncenter=2, prior=prior, family=fam, seed=500 + k,
                             sigma=0.01))
    return out


def _batch(cases, flags=None):
    from paper_1203_4587_amd.api import Batch, Slice
    dev = [c.device() for c in cases]
    slices = [Slice(coil, mask, prior, MU, RHO, 0 if flags is None else flags[k])
              for k, ((coil, mask, _), (_, prior)) in enumerate(zip(dev, SMALL))]
    return Batch(slices), [y for _, _, y in dev], dev


def test_small_uneven_batch_matches_plain_and_oracle():
    from paper_1203_4587_amd.api import Plan
    cases = _small_cases()
    batch, ys, dev = _batch(cases)
    iters = 20
    xs = batch.solve(ys, LAMS, iters)
    torch.cuda.synchronize()
    for k, (case, ((_, prior))) in enumerate(zip(cases, SMALL)):
        coil, mask, y = dev[k]
        plain = Plan(coil, mask, MU, prior=prior, mu_ratio=RHO).solve(y, LAMS[k], iters)
        assert torch.equal(xs[k], plain), k
        ref = O.solve(case.y, case.coil, case.mask, prior, LAMS[k], MU, RHO, iters)
        err = rel_l2(xs[k].cpu().numpy(), ref["x"])
        print(SMALL[k], "rel_l2", err)
        assert err < TOL


@pytest.mark.parametrize("count", [1, 2, 3])
def test_batches_of_few_slices_match_plain(count):
    """The slices are dealt to (at most) two chains of the batch graph: one
    slice, one slice per chain, and a chain of two beside a chain of one all
    solve every slice bit for bit as a plain solve does."""
    from paper_1203_4587_amd.api import Batch, Plan, Slice
    cases = _small_cases()[:count]
    dev = [c.device() for c in cases]
    batch = Batch([Slice(coil, mask, prior, MU, RHO, 0) for (coil, mask, _), (_, prior) in zip(dev, SMALL)])
    ys = [y for _, _, y in dev]
    bufs = [torch.empty(batch.image_shape(k), dtype=torch.complex64, device="cuda") for k in range(count)]
    xs = [t.clone() for t in batch.solve(ys, LAMS[:count], 9, outs=bufs)]
    xs2 = batch.solve(ys, LAMS[:count], 9, outs=bufs)   # the same pointers: a replay
    for k in range(count):
        coil, mask, y = dev[k]
        plain = Plan(coil, mask, MU, prior=SMALL[k][1], mu_ratio=RHO).solve(y, LAMS[k], 9)
        assert torch.equal(xs[k], plain), k
        assert torch.equal(xs2[k], plain), k


def test_batch_graph_replay_tracks_data_and_rerecords():
    """A replay reads the current contents of the same buffers; new buffers,
    lambdas or iteration counts record the graph again.  Every replay is
    checked against plain solves, with eager work in between."""
    from paper_1203_4587_amd.api import Plan
    cases = _small_cases()
    batch, ys, dev = _batch(cases)
    plans = [Plan(c, m, MU, prior=p, mu_ratio=RHO) for (c, m, _), (_, p) in zip(dev, SMALL)]
    outs = [torch.empty(batch.image_shape(k), dtype=torch.complex64, device="cuda") for k in range(len(SMALL))]
    for rep in range(3):
        ys[1].mul_(1.5)  # same buffer, new data
        batch.solve(ys, LAMS, 12, outs=outs)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for k in range(len(SMALL)):
            assert torch.equal(outs[k], plans[k].solve(ys[k], LAMS[k], 12)), (rep, k)
    lams2 = [v * 2 for v in LAMS]
    xs = batch.solve(ys, lams2, 7)            # new lambdas, count and outputs
    for k in range(len(SMALL)):
        assert torch.equal(xs[k], plans[k].solve(ys[k], lams2[k], 7)), k
    xs0 = batch.solve(ys, LAMS, 0)            # zero iterations: H'y
    for k in range(len(SMALL)):
        assert torch.equal(xs0[k], plans[k].solve(ys[k], LAMS[k], 0)), k
    del junk


def test_batch_with_per_slice_forms():
    """Slices may carry different execution forms (column-resident, each
    x-update form); a flag change through the slice's plan re-records."""
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    cases = _small_cases()
    forms = [_lib.CS_FLAG_COLUMN_RESIDENT, _lib.CS_FLAG_XU_GROUP, 0, _lib.CS_FLAG_XU_WAVE,
             _lib.CS_FLAG_COLUMN_RESIDENT, _lib.CS_FLAG_XU_GROUP]
    batch, ys, dev = _batch(cases, forms)
    plain = [Plan(c, m, MU, prior=p, mu_ratio=RHO).solve(y, LAMS[k], 15)
             for k, ((c, m, y), (_, p)) in enumerate(zip(dev, SMALL))]
    xs = batch.solve(ys, LAMS, 15)
    for k in range(len(SMALL)):
        assert torch.equal(xs[k], plain[k]), k
    batch.plan(0).flags = _lib.CS_FLAG_XU_WAVE
    batch.plan(1).flags = _lib.CS_FLAG_COLUMN_RESIDENT
    xs = batch.solve(ys, LAMS, 15)
    for k in range(len(SMALL)):
        assert torch.equal(xs[k], plain[k]), k


def test_batch_replays_after_a_slice_plan_solved_at_another_mu():
    """A slice's plan used on its own at another mu refactors in place; the
    next batch solve must record again with that mu (the recorded kernels carry
    mu) and equal a plain plan built with it.  New FFT tiles re-record too."""
    from paper_1203_4587_amd.api import Plan
    cases = _small_cases()
    batch, ys, dev = _batch(cases)
    iters = 10
    xs = batch.solve(ys, LAMS, iters)           # records with mu = MU
    torch.cuda.synchronize()
    mu2 = 0.37
    for k in (0, 1):
        batch.plan(k).solve(ys[k], LAMS[k], 3, mu=mu2)   # refactors slice k's plan for mu2
    xs = batch.solve(ys, LAMS, iters)
    for k in range(len(SMALL)):
        coil, mask, y = dev[k]
        mu_k = mu2 if k in (0, 1) else MU
        plain = Plan(coil, mask, mu_k, prior=SMALL[k][1], mu_ratio=RHO).solve(y, LAMS[k], iters)
        assert torch.equal(xs[k], plain), k
    case = cases[0]
    ref = O.solve(case.y, case.coil, case.mask, SMALL[0][1], LAMS[0], mu2, RHO, iters)
    assert rel_l2(xs[0].cpu().numpy(), ref["x"]) < TOL
    cw, rb = batch.plan(2).fft_tiles
    batch.plan(2).fft_tiles = (max(1, cw // 2), max(1, rb // 2))
    xs2 = batch.solve(ys, LAMS, iters)
    for k in range(len(SMALL)):
        assert torch.equal(xs2[k], xs[k]), k


@pytest.mark.parametrize("shape,prior", [((128, 16, 16, 3), "tv"), ((192, 12, 24, 3), "dft"),
                                         ((12, 8, 6, 2), "tv"), ((256, 8, 8, 2), "dft"),
                                         # two blocks per wave (n = 64, 192), odd block counts
                                         ((64, 9, 3, 2), "tv"), ((192, 3, 3, 2), "tv"), ((64, 12, 5, 2), "dft")],
                         ids=str)
def test_xupdate_forms_are_bit_identical(shape, prior):
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    nv, nh, nt, nc = shape
    fam = "cardiac" if prior == "tv" else "periodic"
    case = make_case(nv, nh, nt, nc, accel=3, ncenter=2, prior=prior, family=fam, seed=nv + 1)
    coil, mask, y = case.device()
    xs = [Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=f).solve(y, 0.02, 10)
          for f in (0, _lib.CS_FLAG_XU_WAVE, _lib.CS_FLAG_XU_GROUP)]
    assert torch.equal(xs[0], xs[1]) and torch.equal(xs[0], xs[2])
    b = torch.randn(nt, nv, nh, dtype=torch.complex64, device="cuda")
    ws = [Plan(coil, mask, MU, prior=prior, mu_ratio=RHO, flags=f).block_inverse(b)
          for f in (_lib.CS_FLAG_XU_WAVE, _lib.CS_FLAG_XU_GROUP)]
    assert torch.equal(ws[0], ws[1])


def test_autotuner_picks_a_form_and_caches_it(tmp_path):
    from paper_1203_4587_amd import _lib
    from paper_1203_4587_amd.api import Plan
    case = make_case(128, 32, 16, 4, accel=4, ncenter=4, prior="tv", seed=11)
    coil, mask, y = case.device()
    ref = Plan(coil, mask, MU, prior="tv", mu_ratio=RHO).solve(y, 0.02, 10)
    plan = Plan(coil, mask, MU, prior="tv", mu_ratio=RHO, flags=_lib.CS_FLAG_NO_REFACTOR)
    cache = str(tmp_path / "tune.json")
    res = plan.tune(y, 0.02, iters=5, cache=cache)
    print(res)
    assert not res["cached"]
    cand = [f for f, _ in res["candidates"]]
    assert len(cand) == 3 and all(ms > 0 for _, ms in res["candidates"])
    best = min(res["candidates"], key=lambda c: c[1])[0]
    assert plan.flags == best and plan.flags & _lib.CS_FLAG_NO_REFACTOR
    assert torch.equal(plan.solve(y, 0.02, 10), ref)   # tuning never changes results
    again = Plan(coil, mask, MU, prior="tv", mu_ratio=RHO)
    res2 = again.tune(y, 0.02, cache=cache)
    assert res2["cached"] and again.flags == best & ~_lib.CS_FLAG_NO_REFACTOR
    # odd nv: the phase form with the row x-update is the only candidate
    odd = make_case(27, 8, 4, 2, prior="tv", seed=12)
    c2, m2, y2 = odd.device()
    p2 = Plan(c2, m2, MU, prior="tv", mu_ratio=RHO)
    assert [f for f, _ in p2.tune(y2, 0.02, iters=3)["candidates"]] == [_lib.CS_FLAG_GRAPH]


@pytest.fixture(scope="module")
def full_batch():
    """The 24-slice uneven batch at full size, solved for 100 iterations in one
    batched launch.  Keeps, per slice, the oracle's inputs and the GPU image."""
    from paper_1203_4587_amd.api import Batch, Slice, to_device
    slices, ys, host = [], [], []
    for s in range(24):
        pr = S.batch_slice(s)
        case = Case(pr)
        host.append((pr, case.y, case.coil, case.mask))
        slices.append(Slice(to_device(case.coil), to_device(case.mask, dtype=torch.uint8), pr.prior, pr.mu,
                            pr.rho))
        ys.append(to_device(case.y))
    print("24 slices drawn", flush=True)
    batch = Batch(slices)
    xs = batch.solve(ys, [h[0].lam for h in host], 100)
    torch.cuda.synchronize()
    out = [(h, x.cpu().numpy()) for h, x in zip(host, xs)]
    batch.close()
    del xs, ys, slices
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("s", range(24))
def test_full_batch_24_uneven_slices_sampled_columns(full_batch, s):
    """Each slice of the batched launch against its own oracle run on two
    sampled columns (100 iterations)."""
    (pr, y, coil, mask), x = full_batch[s]
    nh = pr.x_true.shape[2]
    cols = np.array(sorted({(7 * s) % nh, nh // 2 + s % 5}))
    ref = O.solve(y, coil, mask, pr.prior, pr.lam, pr.mu, pr.rho, pr.iters, cols=cols)
    err = rel_l2(x[:, :, cols], ref["x"])
    print("slice", s, pr.x_true.shape, pr.prior, "sampled rel_l2", err)
    assert err < TOL

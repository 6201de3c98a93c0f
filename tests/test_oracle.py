"""Pins for the FP64 oracle: each check compares it with something other than
itself (a brute-force definition, a closed form, an invariant, an independent
solver), chosen so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them."""
import numpy as np
import pytest
import scipy.optimize

import oracle as O
from paper_1203_4587_amd import synthetic as S


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def tiny_problem(rng, nt=3, nv=6, nh=4, nc=2, full=False, sos=False):
    coil = crandn(rng, nc, nv, nh)
    if sos:
        coil = coil / np.sqrt((np.abs(coil) ** 2).sum(0))
    if full:
        mask = np.ones((nt, nv), np.uint8)
    else:
        mask = (rng.random((nt, nv)) < 0.5).astype(np.uint8)
        mask[:, 0] = 1
    return coil, mask


def brute_forward(x, coil, mask):
    """Direct double sum over pixels: y[t,c,ky,kx] = mask[t,ky] *
    sum_{j,i} s[c,j,i] x[t,j,i] exp(-2 pi i (ky j / nv + kx i / nh)) / sqrt(nv nh)."""
    nt, nv, nh = x.shape
    nc = coil.shape[0]
    y = np.zeros((nt, nc, nv, nh), complex)
    for t in range(nt):
        for c in range(nc):
            img = coil[c] * x[t]
            for ky in range(nv):
                if not mask[t, ky]:
                    continue
                for kx in range(nh):
                    acc = 0j
                    for j in range(nv):
                        for i in range(nh):
                            acc += img[j, i] * np.exp(-2j * np.pi * (ky * j / nv + kx * i / nh))
                    y[t, c, ky, kx] = acc / np.sqrt(nv * nh)
    return y


def dense_H(coil, mask):
    """Dense matrix of H built column by column from ``brute_forward`` (no FFT)."""
    nt = mask.shape[0]
    nc, nv, nh = coil.shape
    n = nt * nv * nh
    cols = []
    for k in range(n):
        e = np.zeros(n, complex)
        e[k] = 1
        cols.append(brute_forward(e.reshape(nt, nv, nh), coil, mask).ravel())
    return np.stack(cols, axis=1)


# ---------------------------------------------------------------- operator H

@pytest.mark.parametrize("nv,nh", [(4, 6), (6, 4), (8, 12), (12, 8)])
def test_forward_matches_bruteforce_dft(rng, nv, nh):
    coil, mask = tiny_problem(rng, nt=2, nv=nv, nh=nh, nc=2)
    x = crandn(rng, 2, nv, nh)
    np.testing.assert_allclose(O.forward(x, coil, mask), brute_forward(x, coil, mask), atol=1e-12)


def test_adjoint_identity(rng):
    coil, mask = tiny_problem(rng, nt=4, nv=12, nh=8, nc=3)
    x = crandn(rng, 4, 12, 8)
    y = crandn(rng, 4, 3, 12, 8)
    lhs = np.vdot(y, O.forward(x, coil, mask))
    rhs = np.vdot(O.adjoint(y, coil, mask), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_adjoint_ignores_unsampled_rows(rng):
    coil, mask = tiny_problem(rng, nt=2, nv=8, nh=4, nc=2)
    y = crandn(rng, 2, 2, 8, 4)
    y2 = y + crandn(rng, 2, 2, 8, 4) * (1 - mask)[:, None, :, None]
    np.testing.assert_allclose(O.adjoint(y, coil, mask), O.adjoint(y2, coil, mask), atol=1e-14)


def test_full_sampling_sos_is_identity(rng):
    coil, mask = tiny_problem(rng, nt=3, nv=8, nh=6, nc=3, full=True, sos=True)
    x = crandn(rng, 3, 8, 6)
    np.testing.assert_allclose(O.adjoint(O.forward(x, coil, mask), coil, mask), x, atol=1e-12)


def test_parseval(rng):
    coil, mask = tiny_problem(rng, nt=2, nv=6, nh=6, nc=1, full=True)
    coil[:] = 1.0
    x = crandn(rng, 2, 6, 6)
    assert np.isclose(np.linalg.norm(O.forward(x, coil, mask)), np.linalg.norm(x), rtol=1e-13)


def test_adjoint_columns_matches_full(rng):
    coil, mask = tiny_problem(rng, nt=3, nv=8, nh=6, nc=2)
    y = crandn(rng, 3, 2, 8, 6)
    cols = [0, 3, 5]
    np.testing.assert_allclose(O.adjoint_columns(y, coil, mask, cols),
                               O.adjoint(y, coil, mask)[:, :, cols], atol=1e-13)


# ------------------------------------------------- block structure of H'H

def test_HtH_is_block_diagonal_with_gram_blocks(rng):
    nt, nv, nh, nc = 2, 6, 3, 2
    coil, mask = tiny_problem(rng, nt=nt, nv=nv, nh=nh, nc=nc)
    H = dense_H(coil, mask)
    HtH = (H.conj().T @ H).reshape(nt, nv, nh, nt, nv, nh)
    for t in range(nt):
        for i in range(nh):
            G = O.gram_block(coil[:, :, i], mask[t])
            np.testing.assert_allclose(HtH[t, :, i, t, :, i], G, atol=1e-12)
    # everything outside the (t, i) blocks vanishes
    off = HtH.copy()
    for t in range(nt):
        for i in range(nh):
            off[t, :, i, t, :, i] = 0
    assert np.abs(off).max() < 1e-12


def test_gram_coil_term_conjugates_the_row_index(rng):
    """Reading of eq. HconjH: the block equals P .* (conj(s_j) s_k) summed over
    coils; the printed s s' (= s_j conj(s_k)) is its transpose-conjugate
    mismatch for complex s and fails."""
    nv, nc = 6, 3
    s = crandn(rng, nc, nv)
    mask = (rng.random(nv) < 0.5).astype(np.uint8)
    mask[0] = 1
    G = O.gram_block(s, mask)
    Fv = O.dft_matrix(nv)
    P = Fv.conj().T @ np.diag(mask.astype(float)) @ Fv
    C_read = sum(np.outer(np.conj(sc), sc) for sc in s)
    C_printed = sum(np.outer(sc, np.conj(sc)) for sc in s)
    np.testing.assert_allclose(G, P * C_read, atol=1e-13)
    assert np.abs(G - P * C_printed).max() > 1e-3


def test_gram_eigenvalues_in_unit_interval_for_sos_maps(rng):
    p = S.make_problem(16, 8, 3, 4, 4, 4, "tv", "ellipses3", 7)
    fac = O.BlockFactor(p.coil, p.mask)
    assert fac.e.min() > -1e-12 and fac.e.max() < 1 + 1e-12


def test_block_solve_residual(rng):
    coil, mask = tiny_problem(rng, nt=3, nv=12, nh=4, nc=3)
    fac = O.BlockFactor(coil, mask)
    b = crandn(rng, 3, 12, 4)
    mu = 0.07
    x = fac.solve(b, mu)
    for t in range(3):
        for i in range(4):
            G = O.gram_block(coil[:, :, i], mask[t])
            r = (mu * np.eye(12) + G) @ x[t, :, i] - b[t, :, i]
            assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b[t, :, i])


def test_block_solve_full_sampling_closed_form(rng):
    coil, mask = tiny_problem(rng, nt=2, nv=8, nh=3, nc=3, full=True, sos=True)
    fac = O.BlockFactor(coil, mask)
    b = crandn(rng, 2, 8, 3)
    np.testing.assert_allclose(fac.solve(b, 0.1), b / 1.1, atol=1e-13)


def test_block_solve_single_unit_coil_closed_form(rng):
    nt, nv, nh = 3, 12, 2
    coil = np.ones((1, nv, nh), complex)
    mask = (rng.random((nt, nv)) < 0.4).astype(np.uint8)
    fac = O.BlockFactor(coil, mask)
    b = crandn(rng, nt, nv, nh)
    mu = 0.2
    ref = np.fft.ifft(np.fft.fft(b, axis=1, norm="ortho") / (mu + mask[:, :, None]),
                      axis=1, norm="ortho")
    np.testing.assert_allclose(fac.solve(b, mu), ref, atol=1e-13)


# ------------------------------------------------------------- shrinkage

def test_soft_closed_form_and_edges():
    tau = 0.5
    a = np.array([3 + 4j, 0.3 + 0.4j, 0j, 0.5 + 0j, -2.0 + 0j, 1j])
    out = O.soft(a, tau)
    np.testing.assert_allclose(out, [(5 - 0.5) * (3 + 4j) / 5, 0, 0, 0, -1.5, 0.5j], atol=1e-15)
    np.testing.assert_allclose(O.soft(a, 0.0), a)


def test_soft_is_the_prox_by_grid_search(rng):
    """soft(a, lambda/(2 mu)) minimises lambda|v| + mu|v - a|^2 (the v-step)."""
    lam, mu = 0.3, 0.8
    g = np.linspace(-2, 2, 801)
    V = g[:, None] + 1j * g[None, :]
    for a in [0.9 + 0.2j, -0.1 + 0.05j, 1.3 - 1.1j]:
        f = lam * np.abs(V) + mu * np.abs(V - a) ** 2
        vbest = V.ravel()[np.argmin(f)]
        assert abs(O.soft(np.array([a]), lam / (2 * mu))[0] - vbest) < 2 * (g[1] - g[0])


# ---------------------------------------------------------- temporal ops

def test_tdiff_adjoint(rng):
    x = crandn(rng, 7, 3, 2)
    v = crandn(rng, 6, 3, 2)
    assert np.isclose(np.vdot(v, O.tdiff(x)), np.vdot(O.tdiff_adj(v), x), rtol=1e-13)


def test_tdiff_matches_paper_matrix():
    """tdiff applied to the identity reproduces the printed D_t (eq. TV),
    stored as a fixture for n_t = 5."""
    import os
    Dm = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "temporal_difference_nt5.txt"))
    nt = Dm.shape[1]
    np.testing.assert_array_equal(O.tdiff(np.eye(nt)), Dm)


@pytest.mark.parametrize("nt", [2, 3, 8, 33])
def test_tv_system_solve(rng, nt):
    rho = 0.5
    Dm = O.tdiff(np.eye(nt))
    T = rho * np.eye(nt) + Dm.T @ Dm
    r = crandn(rng, nt, 4)
    m = O.tv_system_solve(r, rho)
    np.testing.assert_allclose(T @ m, r, atol=1e-12)
    # DCT-II diagonalisation: eigenvalues rho + 2 - 2 cos(pi k / nt)
    ev = np.sort(np.linalg.eigvalsh(T))
    np.testing.assert_allclose(ev, np.sort(rho + 2 - 2 * np.cos(np.pi * np.arange(nt) / nt)), atol=1e-12)


@pytest.mark.parametrize("nt", [1, 2, 5, 16])
def test_tv_normal_solve_dense(rng, nt):
    """(a D'D + b I) m = r, with D'D formed from the printed D_t by dense
    matrix products (the fixture of eq. TV extended to nt frames)."""
    a, b = 2.5, 0.3
    Dm = np.zeros((nt - 1, nt))
    for t in range(nt - 1):
        Dm[t, t], Dm[t, t + 1] = -1.0, 1.0
    r = crandn(rng, nt, 3)
    m = O.tv_normal_solve(r, a, b)
    np.testing.assert_allclose((a * Dm.T @ Dm + b * np.eye(nt)) @ m, r, atol=1e-12)
    # the Algorithm 2 form divided through by mu_1 is the same system
    np.testing.assert_allclose(O.tv_system_solve(r, b / a), a * m, atol=1e-12)


def test_tdft_unitary_and_bruteforce(rng):
    nt = 6
    z = crandn(rng, nt, 2)
    F = np.array([[np.exp(-2j * np.pi * f * t / nt) for t in range(nt)] for f in range(nt)]) / np.sqrt(nt)
    np.testing.assert_allclose(O.tdft(z), F @ z, atol=1e-13)
    np.testing.assert_allclose(O.tdft_adj(O.tdft(z)), z, atol=1e-13)


# ------------------------------------------------ tight-frame inverse (Sec. IV-A)

def test_tight_frame_inverse_identity(rng):
    n, m, p, mu = 5, 4, 8, 0.3
    H = crandn(rng, m, n)
    Q, _ = np.linalg.qr(crandn(rng, p, n))       # Psi with Psi' Psi = I, Psi Psi' != I
    Psi = Q
    I_p, I_n = np.eye(p), np.eye(n)
    lhs = np.linalg.inv(mu * I_p + Psi @ H.conj().T @ H @ Psi.conj().T)
    final = I_p / mu - Psi @ Psi.conj().T / mu + Psi @ np.linalg.inv(mu * I_n + H.conj().T @ H) @ Psi.conj().T
    np.testing.assert_allclose(lhs, final, atol=1e-12)
    # first line of the derivation as printed lacks 1/mu on the second term
    printed = I_p / mu - Psi @ H.conj().T @ np.linalg.inv(mu * np.eye(m) + H @ H.conj().T) @ H @ Psi.conj().T
    fixed = I_p / mu - Psi @ H.conj().T @ np.linalg.inv(mu * np.eye(m) + H @ H.conj().T) @ H @ Psi.conj().T / mu
    np.testing.assert_allclose(lhs, fixed, atol=1e-12)
    assert np.abs(lhs - printed).max() > 1e-2


def test_union_frame_is_tight_and_overcomplete(rng):
    """tframe = [I; F_t] / sqrt(2): Psi'Psi = I (tight), Psi Psi' != I but a
    projection; its matrix equals the stacked identity and brute-force DFT."""
    nt = 6
    z = crandn(rng, nt, 3, 2)
    np.testing.assert_allclose(O.tframe_adj(O.tframe(z)), z, atol=1e-14)
    P = np.stack([O.tframe(np.eye(nt)[:, k][:, None, None])[:, 0, 0] for k in range(nt)], axis=1)
    F = np.exp(-2j * np.pi * np.outer(np.arange(nt), np.arange(nt)) / nt) / np.sqrt(nt)
    np.testing.assert_allclose(P, np.vstack([np.eye(nt), F]) / np.sqrt(2), atol=1e-14)
    G = P @ P.conj().T
    assert np.abs(G - np.eye(2 * nt)).max() > 0.1          # overcomplete
    np.testing.assert_allclose(G @ G, G, atol=1e-14)        # orthogonal projection
    w = crandn(rng, 2 * nt, 3, 2)
    np.testing.assert_allclose(np.vdot(O.tframe(z), w), np.vdot(z, O.tframe_adj(w)), atol=1e-13)


def test_synthesis_with_union_frame_reaches_kkt_point():
    """Algorithm 1 with the overcomplete frame converges to a minimiser of
    lambda ||w||_1 + ||y - H Psi' w||^2: with g = 2 Psi H'(H Psi' w - y),
    g = -lambda w/|w| on the support and |g| <= lambda elsewhere."""
    from tests.helpers import make_case
    case = make_case(8, 4, 6, 2, accel=2, ncenter=2, prior="dft", family="periodic", seed=3, sigma=0.02)
    lam, mu = 0.05, 0.5
    fac = O.BlockFactor(case.coil, case.mask)
    Hy = O.adjoint(case.y, case.coil, case.mask)
    w = O.admm_synthesis(Hy, fac, lam, mu, 3000, psi=O.tframe, psi_adj=O.tframe_adj)["w"]
    x = O.tframe_adj(w)
    g = 2 * O.tframe(O.adjoint(O.forward(x, case.coil, case.mask), case.coil, case.mask) - Hy)
    nz = np.abs(w) > 1e-9
    assert 0.0 < nz.mean() < 0.5                      # a sparse, non-trivial solution
    assert np.abs(g[nz] + lam * w[nz] / np.abs(w[nz])).max() < 1e-10
    assert np.abs(g[~nz]).max() <= lam * (1 + 1e-9)


def test_synthesis_with_overcomplete_frame_solves_w_subproblem(rng):
    """One Algorithm 1 w-step with an overcomplete tight frame equals the
    minimiser of ||y - H Psi' w||^2 + mu ||w - v - d||^2 (dense normal equations)."""
    nt, nv, nh, nc = 3, 4, 2, 2
    coil, mask = tiny_problem(rng, nt=nt, nv=nv, nh=nh, nc=nc)
    y = crandn(rng, nt, nc, nv, nh) * mask[:, None, :, None]
    fac = O.BlockFactor(coil, mask)
    # temporal frame: [Id; DFT] / sqrt(2) stacked along frames (6 rows, Psi'Psi = I)
    psi, psi_adj = O.tframe, O.tframe_adj
    Hy = O.adjoint(y, coil, mask)
    lam, mu = 0.05, 0.4
    st = O.admm_synthesis(Hy, fac, lam, mu, 1, psi=psi, psi_adj=psi_adj)
    # dense check of the w-step from w0 = Psi H'y, d0 = 0
    H = dense_H(coil, mask)
    n = nt * nv * nh
    P = np.stack([psi(np.eye(n)[:, k].reshape(nt, nv, nh)).ravel() for k in range(n)], axis=1)
    w0 = P @ Hy.ravel()
    v1 = O.soft(w0, lam / (2 * mu))
    A = P @ H.conj().T @ H @ P.conj().T + mu * np.eye(P.shape[0])
    w1 = np.linalg.solve(A, P @ H.conj().T @ y.ravel() + mu * v1)
    np.testing.assert_allclose(st["w"].ravel(), w1, atol=1e-11)
    np.testing.assert_allclose(st["v"].ravel(), v1, atol=1e-12)
    d1 = -(w1 - v1)
    np.testing.assert_allclose(st["d"].ravel(), d1, atol=1e-11)


# ------------------------------------------------- whole-algorithm pins

def small_tv_case(rng, sigma=0.01):
    p = S.make_problem(8, 4, 6, 3, 2, 2, "tv", "ellipses3", 11, sigma=sigma)
    y = O.measure(p)
    return p, y


def test_tv_converges_to_kkt_point(rng):
    p, y = small_tv_case(rng)
    lam, mu, rho = 0.02, 0.1, 0.5
    mu1 = mu / rho
    tau = lam / (2 * mu1)
    st = O.solve(y, p.coil, p.mask, "tv", lam, mu, rho, 3000)
    x, d1 = st["x"], st["d1"]
    grad = 2 * O.adjoint(O.forward(x, p.coil, p.mask) - y, p.coil, p.mask) + 2 * mu1 * O.tdiff_adj(d1)
    assert np.linalg.norm(grad) < 1e-9 * np.linalg.norm(O.adjoint(y, p.coil, p.mask))
    assert np.abs(d1).max() <= tau * (1 + 1e-9)
    Dx = O.tdiff(x)
    on = np.abs(Dx) > 1e-6
    np.testing.assert_allclose(d1[on], tau * Dx[on] / np.abs(Dx[on]), atol=1e-7)
    np.testing.assert_allclose(st["m"], x, atol=1e-10)


def split_bregman_dense(H, y, R, lam, mu, iters):
    """P1 (Sec. III, eqs. admm_bregman_1..3) with an exact dense inverse."""
    x = H.conj().T @ y
    d = np.zeros(R.shape[0], complex)
    Minv = np.linalg.inv(mu * R.conj().T @ R + H.conj().T @ H)
    Hy = H.conj().T @ y
    for _ in range(iters):
        v = O.soft(R @ x - d, lam / (2 * mu))
        x = Minv @ (Hy + mu * R.conj().T @ (v + d))
        d = d - (R @ x - v)
    return x


def test_tv_agrees_with_dense_split_bregman(rng):
    p, y = small_tv_case(rng)
    lam, mu, rho = 0.02, 0.1, 0.5
    nt, nv, nh, nc = p.shape
    st = O.solve(y, p.coil, p.mask, "tv", lam, mu, rho, 3000)
    H = dense_H(p.coil, p.mask)
    # the block Grams are nonsingular here, so the minimiser is unique
    assert np.linalg.matrix_rank(H) == nt * nv * nh
    n = nt * nv * nh
    R = np.stack([O.tdiff(np.eye(n)[:, k].reshape(nt, nv, nh)).ravel() for k in range(n)], axis=1)
    x_sb = split_bregman_dense(H, y.ravel(), R, lam, 0.05, 6000).reshape(nt, nv, nh)
    np.testing.assert_allclose(st["x"], x_sb, atol=1e-7)
    J1 = O.objective_tv(st["x"], y, p.coil, p.mask, lam)
    J2 = O.objective_tv(x_sb, y, p.coil, p.mask, lam)
    assert abs(J1 - J2) <= 1e-12 * J1


def test_dft_full_sampling_closed_form(rng):
    """Full sampling with SoS maps: H'H = I and Algorithm 1 converges to
    Psi' soft(Psi H'y, lambda/2)."""
    p = S.make_problem(8, 6, 5, 3, 1, 8, "dft", "periodic", 21, sigma=0.01)
    p.mask[:] = 1
    y = O.measure(p)
    lam, mu = 0.05, 0.3
    st = O.solve(y, p.coil, p.mask, "dft", lam, mu, 0.5, 400)
    Hy = O.adjoint(y, p.coil, p.mask)
    ref = O.tdft_adj(O.soft(O.tdft(Hy), lam / 2))
    np.testing.assert_allclose(st["x"], ref, atol=1e-12)


def test_tv_full_sampling_real_is_1d_tv_denoising():
    """Full sampling, SoS maps, real data: the problem is per-pixel 1D TV
    denoising min 1/2||x - z||^2 + (lambda/2) TV(x), z = H'y.  Reference: its
    box-constrained dual solved by L-BFGS-B, x = z - D'u."""
    rng = np.random.default_rng(5)
    nt, nv, nh, nc = 7, 4, 2, 2
    coil = np.abs(rng.standard_normal((nc, nv, nh))) + 0.2
    coil = coil / np.sqrt((coil ** 2).sum(0))
    mask = np.ones((nt, nv), np.uint8)
    x0 = np.cumsum(rng.standard_normal((nt, nv, nh)), axis=0)
    y = O.forward(x0, coil, mask)
    lam, mu, rho = 0.8, 0.5, 0.5
    st = O.solve(y, coil, mask, "tv", lam, mu, rho, 4000)
    z = O.adjoint(y, coil, mask).real
    Dm = O.tdiff(np.eye(nt))
    for j in range(nv):
        for i in range(nh):
            zz = z[:, j, i]

            def f(u):
                r = zz - Dm.T @ u
                return 0.5 * r @ r, -(Dm @ r)
            res = scipy.optimize.minimize(f, np.zeros(nt - 1), jac=True, method="L-BFGS-B",
                                          bounds=[(-lam / 2, lam / 2)] * (nt - 1),
                                          options=dict(ftol=1e-15, gtol=1e-13, maxiter=10000))
            xref = zz - Dm.T @ res.x
            np.testing.assert_allclose(st["x"][:, j, i], xref, atol=1e-7)


def test_tv_lambda_zero_full_sampling_fixed_point(rng):
    p = S.make_problem(8, 4, 4, 2, 1, 8, "tv", "ellipses3", 31)
    p.mask[:] = 1
    y = O.measure(p)
    st = O.solve(y, p.coil, p.mask, "tv", 0.0, 0.1, 0.5, 7)
    np.testing.assert_allclose(st["x"], O.adjoint(y, p.coil, p.mask), atol=1e-13)


def test_column_subset_equals_full(rng):
    p = S.make_problem(8, 6, 4, 2, 2, 2, "tv", "cardiac", 41)
    y = O.measure(p)
    full = O.solve(y, p.coil, p.mask, "tv", 0.01, 0.1, 0.5, 20)
    sub = O.solve(y, p.coil, p.mask, "tv", 0.01, 0.1, 0.5, 20, cols=[1, 4])
    np.testing.assert_allclose(sub["x"], full["x"][:, :, [1, 4]], atol=1e-13)
    fd = O.solve(y, p.coil, p.mask, "dft", 0.01, 0.1, 0.5, 20)
    sd = O.solve(y, p.coil, p.mask, "dft", 0.01, 0.1, 0.5, 20, cols=[0, 5])
    np.testing.assert_allclose(sd["x"], fd["x"][:, :, [0, 5]], atol=1e-13)


def test_resume_equals_uninterrupted(rng):
    p = S.make_problem(8, 4, 5, 2, 2, 2, "tv", "cardiac", 51)
    y = O.measure(p)
    fac = O.BlockFactor(p.coil, p.mask)
    Hy = O.adjoint(y, p.coil, p.mask)
    a = O.admm_analysis(Hy, fac, 0.01, 0.1, 0.5, 50)
    b = O.admm_analysis(Hy, fac, 0.01, 0.1, 0.5, 25)
    b = O.admm_analysis(Hy, fac, 0.01, 0.1, 0.5, 25, state=b)
    for k in ("x", "m", "d1", "d2"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-15)
    a = O.admm_synthesis(Hy, fac, 0.01, 0.1, 30)
    b = O.admm_synthesis(Hy, fac, 0.01, 0.1, 10)
    b = O.admm_synthesis(Hy, fac, 0.01, 0.1, 20, state=b)
    for k in ("x", "w", "v", "d"):
        np.testing.assert_allclose(a[k], b[k], atol=1e-15)


def test_delta_literal_values():
    """Delta(k) = (J(k-1) - J(k)) / J(k) (eq. r_ratio) on literal values: the
    numerator is the drop from the previous to the current objective and the
    denominator is the current one, so a rise gives a negative ratio."""
    assert O.delta(3.0, 2.0) == 0.5                 # drop of 1 over J(k) = 2 (not over J(k-1) = 3)
    assert O.delta(2.0, 3.0) == -1.0 / 3.0          # J rises: negative
    assert O.delta(5.0, 5.0) == 0.0
    assert O.delta(1.001, 1.0) == pytest.approx(0.001, rel=1e-12)
    # sign and denominator: (J(k) - J(k-1)) / J(k) or a division by J(k-1) both fail here
    assert O.delta(4.0, 1.0) == 3.0


def test_delta_and_objective_decrease():
    p = S.CONFIGS["tv64"]()
    y = O.measure(p)
    Js = []
    O.solve(y, p.coil, p.mask, "tv", p.lam, p.mu, p.rho, 0)  # warm path
    fac = O.BlockFactor(p.coil, p.mask)
    Hy = O.adjoint(y, p.coil, p.mask)
    O.admm_analysis(Hy, fac, p.lam, p.mu, p.rho, 30,
                    callback=lambda k, x: Js.append(O.objective_tv(x, y, p.coil, p.mask, p.lam)))
    J0 = O.objective_tv(Hy, y, p.coil, p.mask, p.lam)
    assert Js[-1] < J0
    d = [O.delta(a, b) for a, b in zip(Js[:-1], Js[1:])]
    assert abs(d[-1]) < abs(d[0])


# ------------------------------------- one iteration = the stated sub-problems

def test_tv_iteration_steps_are_the_stated_argmins(rng):
    """From a random state, one Algorithm 2 iteration must produce, in order:
    v = prox of the l1 term at D m + d1 (old m), m minimising
    mu1||v - D m - d1||^2 + mu2||m - x - d2||^2 (old x, d2), x minimising
    ||y - Hx||^2 + mu2||m - x - d2||^2 (new m, old d2), d1 = d1 - (v - D m)
    (new m) and d2 = d2 - (m - x) (new m, x).  Checked with dense matrices."""
    nt, nv, nh, nc = 3, 4, 2, 2
    coil, mask = tiny_problem(rng, nt=nt, nv=nv, nh=nh, nc=nc)
    y = crandn(rng, nt, nc, nv, nh) * mask[:, None, :, None]
    lam, mu, rho = 0.3, 0.2, 0.25
    mu1 = mu / rho
    st0 = {"x": crandn(rng, nt, nv, nh), "m": crandn(rng, nt, nv, nh),
           "d1": 0.1 * crandn(rng, nt - 1, nv, nh), "d2": 0.1 * crandn(rng, nt, nv, nh)}
    fac = O.BlockFactor(coil, mask)
    Hy = O.adjoint(y, coil, mask)
    st1 = O.admm_analysis(Hy, fac, lam, mu, rho, 1, state=st0)
    n = nt * nv * nh
    H = dense_H(coil, mask)
    R = np.stack([O.tdiff(np.eye(n)[:, k].reshape(nt, nv, nh)).ravel() for k in range(n)], axis=1)
    m0, d10, x0, d20 = (st0[k].ravel() for k in ("m", "d1", "x", "d2"))
    v = O.soft(R @ m0 + d10, lam / (2 * mu1))
    m1 = np.linalg.solve(mu1 * R.T @ R + mu * np.eye(n), mu1 * R.T @ (v - d10) + mu * (x0 + d20))
    x1 = np.linalg.solve(H.conj().T @ H + mu * np.eye(n), H.conj().T @ y.ravel() + mu * (m1 - d20))
    np.testing.assert_allclose(st1["m"].ravel(), m1, atol=1e-12)
    np.testing.assert_allclose(st1["x"].ravel(), x1, atol=1e-12)
    np.testing.assert_allclose(st1["d1"].ravel(), d10 - (v - R @ m1), atol=1e-12)
    np.testing.assert_allclose(st1["d2"].ravel(), d20 - (m1 - x1), atol=1e-12)


def test_dft_iteration_steps_are_the_stated_argmins(rng):
    nt, nv, nh, nc = 4, 4, 2, 2
    coil, mask = tiny_problem(rng, nt=nt, nv=nv, nh=nh, nc=nc)
    y = crandn(rng, nt, nc, nv, nh) * mask[:, None, :, None]
    lam, mu = 0.3, 0.2
    st0 = {"w": crandn(rng, nt, nv, nh), "v": crandn(rng, nt, nv, nh),
           "d": 0.1 * crandn(rng, nt, nv, nh)}
    fac = O.BlockFactor(coil, mask)
    Hy = O.adjoint(y, coil, mask)
    st1 = O.admm_synthesis(Hy, fac, lam, mu, 1, state=st0)
    n = nt * nv * nh
    H = dense_H(coil, mask)
    P = np.stack([O.tdft(np.eye(n)[:, k].reshape(nt, nv, nh)).ravel() for k in range(n)], axis=1)
    w0, d0 = st0["w"].ravel(), st0["d"].ravel()
    v = O.soft(w0 - d0, lam / (2 * mu))
    HP = H @ P.conj().T
    w1 = np.linalg.solve(HP.conj().T @ HP + mu * np.eye(n), HP.conj().T @ y.ravel() + mu * (v + d0))
    np.testing.assert_allclose(st1["v"].ravel(), v, atol=1e-12)
    np.testing.assert_allclose(st1["w"].ravel(), w1, atol=1e-12)
    np.testing.assert_allclose(st1["d"].ravel(), d0 - (w1 - v), atol=1e-12)
    np.testing.assert_allclose(st1["x"].ravel(), P.conj().T @ w1, atol=1e-12)


def test_objectives_match_dense_definitions(rng):
    """J of eqs. L1an_pri / L1unconst from dense matrices built without FFTs."""
    nt, nv, nh, nc = 3, 4, 2, 2
    coil, mask = tiny_problem(rng, nt=nt, nv=nv, nh=nh, nc=nc)
    y = crandn(rng, nt, nc, nv, nh) * mask[:, None, :, None]
    x = crandn(rng, nt, nv, nh)
    lam = 0.37
    H = dense_H(coil, mask)
    r = y.ravel() - H @ x.ravel()
    Dm = np.zeros((nt - 1, nt))
    for t in range(nt - 1):
        Dm[t, t], Dm[t, t + 1] = -1, 1
    Dx = np.einsum("st,tji->sji", Dm, x)
    J_tv = lam * np.abs(Dx).sum() + np.vdot(r, r).real
    assert np.isclose(O.objective_tv(x, y, coil, mask, lam), J_tv, rtol=1e-13)
    Fm = np.array([[np.exp(-2j * np.pi * f * t / nt) for t in range(nt)] for f in range(nt)]) / np.sqrt(nt)
    Px = np.einsum("ft,tji->fji", Fm, x)
    J_dft = lam * np.abs(Px).sum() + np.vdot(r, r).real
    assert np.isclose(O.objective_dft(x, y, coil, mask, lam), J_dft, rtol=1e-13)
    # synthesis objective at coefficients w of the frame Psi = [I; F] / sqrt(2)
    # (2 nt coefficient frames, identity part first): x = Psi' w from the dense
    # matrices, and the l1 term on w itself
    w = crandn(rng, 2 * nt, nv, nh)
    Psi = np.vstack([np.eye(nt), Fm]) / np.sqrt(2.0)
    xw = np.einsum("kt,kji->tji", Psi.conj(), w)
    rw = y.ravel() - H @ xw.ravel()
    J_frame = lam * np.abs(w).sum() + np.vdot(rw, rw).real
    assert np.isclose(O.objective_synthesis(w, y, coil, mask, lam, psi_adj=O.tframe_adj), J_frame, rtol=1e-13)
    # with the orthonormal DFT it is the DFT objective at x = Psi' w
    assert np.isclose(O.objective_synthesis(O.tdft(x), y, coil, mask, lam), J_dft, rtol=1e-13)

"""FP64 reference gradients of unrolled Algorithm 2 (temporal TV) and Algorithm 1
(temporal DFT).

TEST INFRASTRUCTURE ONLY, like ``reference.py``: imported only by the test
suite, the smoke check and the benchmark's CPU-baseline leg, and sharing no
code with the HIP path.

What is differentiated.  K iterations of Algorithm 2 (Sec. IV-B) from its
initialisation x = m = H'y, d1 = d2 = 0, with mu = mu_2, rho = mu_2/mu_1 held
fixed (Sec. V chooses the ratio) and tau = lambda / (2 mu_1).  One iteration,
in the algorithm's order, with D = D_t of eq. TV and T = rho I + D'D:

    a   = D m + d1
    v   = soft(a, tau)                              (Sec. III)
    r   = D'(v - d1) + rho (x + d2)
    m'  = T^{-1} r
    b   = H'y + mu (m' - d2)
    x'  = (mu I + H'H)^{-1} b                       (eq. eigen_mu)
    d1' = d1 - (v - D m')
    d2' = d2 - (m' - x')

The output is x_K; a loss L(x_K) enters through its gradient g = dL/dRe x_K
+ i dL/dIm x_K (the convention of torch.autograd for complex tensors).  The
reverse sweep below applies the transposed Jacobian of each line above, last
line first, with every quantity of the forward pass stored (no
checkpointing here).  For a complex-linear map z' = M z the adjoint is
M' (conjugate transpose); soft() is only real-differentiable and is handled
through its real 2x2 Jacobian; derivatives with respect to the real scalars
use dL/ds = Re sum conj(g_z) dz/ds.  mu enters in three places: tau, the
right-hand side b, and the inverse (mu I + H'H)^{-1}, whose derivative is
-(mu I + H'H)^{-2} (taken here from the eigendecomposition).  Since
H'y = A'(y) is complex-linear in y, dL/dy = A(dL/dH'y).

Derivatives do not exist where some |a| equals tau exactly; elsewhere the
unrolled map is smooth.
"""
from __future__ import annotations

import numpy as np

from .reference import (BlockFactor, adjoint_columns, forward, soft, tdft, tdft_adj, tdiff, tdiff_adj,
                        tv_system_solve)


def _rdot(u: np.ndarray, w: np.ndarray) -> float:
    """Re sum conj(u) w: the real inner product of complex arrays."""
    return float(np.real(np.vdot(u, w)))


def soft_vjp(a: np.ndarray, tau: float, gv: np.ndarray):
    """Transposed Jacobian of v = soft(a, tau) applied to gv, and dL/dtau.

    On |a| > tau, with a written as the real 2-vector (Re a, Im a) and r = |a|,
    v = (1 - tau / r) a, so dv/da = (1 - tau/r) I + (tau / r^3) a a^T (a
    symmetric 2x2 matrix) and dv/dtau = -a / r.  On |a| < tau, v = 0 nearby."""
    a = np.asarray(a, dtype=np.complex128)
    r = np.abs(a)
    on = r > tau
    ga = np.zeros_like(a)
    ar, ai = a.real[on], a.imag[on]
    gr, gi = gv.real[on], gv.imag[on]
    ro = r[on]
    c = 1.0 - tau / ro
    k = tau / ro ** 3
    # [[c + k ar^2, k ar ai], [k ar ai, c + k ai^2]] @ (gr, gi)
    out_r = (c + k * ar * ar) * gr + (k * ar * ai) * gi
    out_i = (k * ar * ai) * gr + (c + k * ai * ai) * gi
    ga[on] = out_r + 1j * out_i
    gtau = float(np.sum(-(ar * gr + ai * gi) / ro))
    return ga, gtau


def unrolled_tv_forward(Hy: np.ndarray, fac: BlockFactor, lam: float, mu: float, rho: float, iters: int):
    """Algorithm 2 for `iters` iterations, returning x_K and every iteration's
    stored quantities (inputs m, d1, x, d2 and a, v, m', b, x')."""
    mu1 = mu / rho
    tau = lam / (2.0 * mu1)
    x = Hy.copy()
    m = x.copy()
    d1 = np.zeros((Hy.shape[0] - 1,) + Hy.shape[1:], dtype=np.complex128)
    d2 = np.zeros_like(Hy)
    tape = []
    for _ in range(iters):
        a = tdiff(m) + d1
        v = soft(a, tau)
        r = tdiff_adj(v - d1) + rho * (x + d2)
        mn = tv_system_solve(r, rho)
        b = Hy + mu * (mn - d2)
        xn = fac.solve(b, mu)
        tape.append(dict(m=m, d1=d1, x=x, d2=d2, a=a, v=v, mn=mn, b=b, xn=xn))
        d1 = d1 - (v - tdiff(mn))
        d2 = d2 - (mn - xn)
        m, x = mn, xn
    return x, tape


def unrolled_tv_grad(Hy: np.ndarray, fac: BlockFactor, lam: float, mu: float, rho: float, iters: int,
                     gx: np.ndarray) -> dict:
    """Reverse sweep of `iters` iterations of Algorithm 2 for the loss gradient
    gx = dL/dx_K.  Returns {"x": x_K, "Hy": dL/dH'y, "lam": dL/dlambda,
    "mu": dL/dmu}.  Arrays have the shape of Hy (nt, nv, k)."""
    mu1 = mu / rho
    tau = lam / (2.0 * mu1)
    xK, tape = unrolled_tv_forward(Hy, fac, lam, mu, rho, iters)
    # adjoints of the state after the last iteration
    gm = np.zeros_like(Hy)
    gxs = np.asarray(gx, dtype=np.complex128).copy()
    gd1 = np.zeros((Hy.shape[0] - 1,) + Hy.shape[1:], dtype=np.complex128)
    gd2 = np.zeros_like(Hy)
    gHy = np.zeros_like(Hy)
    gtau = 0.0
    gmu = 0.0
    for st in reversed(tape):
        # d2' = d2 - m' + x'
        n_gd2 = gd2.copy()
        g_mn = gm - gd2
        g_xn = gxs + gd2
        # d1' = d1 - v + D m'
        n_gd1 = gd1.copy()
        g_v = -gd1
        g_mn = g_mn + tdiff_adj(gd1)
        # x' = (mu I + H'H)^{-1} b: the inverse is Hermitian; d/dmu = -(.)^{-2}
        g_b = fac.solve(g_xn, mu)
        gmu += _rdot(g_xn, -fac.solve(fac.solve(st["b"], mu), mu))
        # b = H'y + mu (m' - d2)
        gHy += g_b
        g_mn = g_mn + mu * g_b
        n_gd2 = n_gd2 - mu * g_b
        gmu += _rdot(g_b, st["mn"] - st["d2"])
        # m' = T^{-1} r, T real symmetric
        g_r = tv_system_solve(g_mn, rho)
        # r = D'(v - d1) + rho (x + d2)
        g_v = g_v + tdiff(g_r)
        n_gd1 = n_gd1 - tdiff(g_r)
        n_gx = rho * g_r
        n_gd2 = n_gd2 + rho * g_r
        # v = soft(a, tau)
        g_a, gt = soft_vjp(st["a"], tau, g_v)
        gtau += gt
        # a = D m + d1
        n_gm = tdiff_adj(g_a)
        n_gd1 = n_gd1 + g_a
        gm, gxs, gd1, gd2 = n_gm, n_gx, n_gd1, n_gd2
    # initialisation x_0 = m_0 = H'y (d1_0 = d2_0 = 0 are constants)
    gHy += gm + gxs
    # tau = lambda rho / (2 mu)
    glam = gtau * rho / (2.0 * mu)
    gmu += gtau * (-lam * rho / (2.0 * mu * mu))
    return {"x": xK, "Hy": gHy, "lam": glam, "mu": gmu}


def unrolled_tv_grad_y(y, coil, mask, lam, mu, rho, iters, gx, cols=None, fac=None) -> dict:
    """dL/dy, dL/dlambda, dL/dmu of L(x_K) for K = iters unrolled iterations of
    Algorithm 2 on data y, given gx = dL/dx_K.

    With `cols`, gx must vanish outside those columns (the image columns i):
    columns never interact, so the sweep runs on them alone, and dL/dH'y is
    zero elsewhere; gx is then passed restricted, shape (nt, nv, len(cols)).
    dL/dy = A(dL/dH'y) is returned at full size (nt, nc, nv, nh), zero on the
    rows a frame does not sample."""
    nt, nv = mask.shape
    nh = coil.shape[2]
    cols = np.arange(nh) if cols is None else np.asarray(cols)
    if fac is None:
        fac = BlockFactor(coil, mask, cols)
    Hy = adjoint_columns(y, coil, mask, cols)
    res = unrolled_tv_grad(Hy, fac, lam, mu, rho, iters, gx)
    gHy = np.zeros((nt, nv, nh), dtype=np.complex128)
    gHy[:, :, cols] = res["Hy"]
    return {"x": res["x"], "y": forward(gHy, coil, mask), "lam": res["lam"], "mu": res["mu"],
            "Hy": res["Hy"]}


def unrolled_tv_loss(y, coil, mask, lam, mu, rho, iters, g, cols=None, fac=None) -> float:
    """L = Re <g, x_K> (sum of conj(g) x_K) for the same unrolled map; used by
    the finite-difference pins."""
    nh = coil.shape[2]
    cols = np.arange(nh) if cols is None else np.asarray(cols)
    if fac is None:
        fac = BlockFactor(coil, mask, cols)
    Hy = adjoint_columns(y, coil, mask, cols)
    xK, _ = unrolled_tv_forward(Hy, fac, lam, mu, rho, iters)
    return _rdot(g, xK)


# --------------------------------------------------------------------------
# Algorithm 1 (synthesis prior, Psi = unitary temporal DFT)
# --------------------------------------------------------------------------
#
# K iterations of Algorithm 1 (Sec. IV-A) from its initialisation w = Psi H'y,
# d = 0, with tau = lambda / (2 mu).  Psi is orthonormal, so the (1/mu)(I -
# Psi Psi') term of the w-update vanishes and one iteration is
#
#     a  = w - d
#     v  = soft(a, tau)
#     u  = Psi'(v + d)
#     b  = H'y + mu u
#     z  = (mu I + H'H)^{-1} b
#     w' = Psi z
#     d' = d - (w' - v)
#
# with output x_K = Psi' w_K (= z_K for K > 0, H'y for K = 0).  The reverse
# sweep follows the same conventions as the one above.


def unrolled_dft_forward(Hy: np.ndarray, fac: BlockFactor, lam: float, mu: float, iters: int):
    """Algorithm 1 for `iters` iterations, returning x_K and every iteration's
    stored quantities (a, u, b, z)."""
    tau = lam / (2.0 * mu)
    w = tdft(Hy)
    d = np.zeros_like(w)
    tape = []
    for _ in range(iters):
        a = w - d
        v = soft(a, tau)
        u = tdft_adj(v + d)
        b = Hy + mu * u
        z = fac.solve(b, mu)
        tape.append(dict(a=a, u=u, b=b, z=z))
        wn = tdft(z)
        d = d - (wn - v)
        w = wn
    return tdft_adj(w), tape


def unrolled_dft_grad(Hy: np.ndarray, fac: BlockFactor, lam: float, mu: float, iters: int,
                      gx: np.ndarray) -> dict:
    """Reverse sweep of `iters` iterations of Algorithm 1 for gx = dL/dx_K.
    Returns {"x": x_K, "Hy": dL/dH'y, "lam": dL/dlambda, "mu": dL/dmu}."""
    tau = lam / (2.0 * mu)
    xK, tape = unrolled_dft_forward(Hy, fac, lam, mu, iters)
    # x_K = Psi' w_K: the adjoint of Psi' is Psi
    gw = tdft(np.asarray(gx, dtype=np.complex128))
    gd = np.zeros_like(gw)
    gHy = np.zeros_like(Hy)
    gtau = 0.0
    gmu = 0.0
    for st in reversed(tape):
        # d' = d - w' + v
        n_gd = gd.copy()
        g_wn = gw - gd
        g_v = gd.copy()
        # w' = Psi z
        g_z = tdft_adj(g_wn)
        # z = (mu I + H'H)^{-1} b: the inverse is Hermitian; d/dmu = -(.)^{-2}
        g_b = fac.solve(g_z, mu)
        gmu += _rdot(g_z, -fac.solve(fac.solve(st["b"], mu), mu))
        # b = H'y + mu u
        gHy += g_b
        g_u = mu * g_b
        gmu += _rdot(g_b, st["u"])
        # u = Psi'(v + d)
        s = tdft(g_u)
        g_v = g_v + s
        n_gd = n_gd + s
        # v = soft(a, tau)
        g_a, gt = soft_vjp(st["a"], tau, g_v)
        gtau += gt
        # a = w - d
        gw = g_a
        gd = n_gd - g_a
    # initialisation w_0 = Psi H'y (d_0 = 0 is a constant)
    gHy += tdft_adj(gw)
    # tau = lambda / (2 mu)
    glam = gtau / (2.0 * mu)
    gmu += gtau * (-lam / (2.0 * mu * mu))
    return {"x": xK, "Hy": gHy, "lam": glam, "mu": gmu}


def unrolled_dft_grad_y(y, coil, mask, lam, mu, iters, gx, cols=None, fac=None) -> dict:
    """dL/dy, dL/dlambda, dL/dmu of L(x_K) for K = iters unrolled iterations of
    Algorithm 1 on data y, given gx = dL/dx_K (column restriction as for
    unrolled_tv_grad_y)."""
    nt, nv = mask.shape
    nh = coil.shape[2]
    cols = np.arange(nh) if cols is None else np.asarray(cols)
    if fac is None:
        fac = BlockFactor(coil, mask, cols)
    Hy = adjoint_columns(y, coil, mask, cols)
    res = unrolled_dft_grad(Hy, fac, lam, mu, iters, gx)
    gHy = np.zeros((nt, nv, nh), dtype=np.complex128)
    gHy[:, :, cols] = res["Hy"]
    return {"x": res["x"], "y": forward(gHy, coil, mask), "lam": res["lam"], "mu": res["mu"],
            "Hy": res["Hy"]}


def unrolled_dft_loss(y, coil, mask, lam, mu, iters, g, cols=None, fac=None) -> float:
    """L = Re <g, x_K> for the unrolled Algorithm 1 map (finite-difference pins)."""
    nh = coil.shape[2]
    cols = np.arange(nh) if cols is None else np.asarray(cols)
    if fac is None:
        fac = BlockFactor(coil, mask, cols)
    Hy = adjoint_columns(y, coil, mask, cols)
    xK, _ = unrolled_dft_forward(Hy, fac, lam, mu, iters)
    return _rdot(g, xK)

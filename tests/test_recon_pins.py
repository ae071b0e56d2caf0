"""Pins of the reconstruction / learned-preconditioner oracle (oracle/recon.py)
against facts that do not come from the oracle itself: library routines for
textbook special cases, closed-form eigenpairs, transposition identities,
finite differences and dense linear algebra."""
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

import oracle
import oracle.recon as R


def _rng(seed=0):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- convolution
def test_conv3x3_matches_scipy_correlate():
    rng = _rng(1)
    B, H, W, ci, co = 2, 7, 9, 3, 4
    x = rng.normal(size=(B, H, W, ci))
    w = rng.normal(size=(9, co, ci))
    y = R.conv3x3(x, w)
    for b in range(B):
        for o in range(co):
            ref = np.zeros((H, W))
            for i in range(ci):
                k = w[:, o, i].reshape(3, 3)      # k[ky][kx] multiplies x[h+ky-1, w+kx-1]
                ref += correlate2d(x[b, :, :, i], k, mode="same", boundary="fill")
            assert np.allclose(y[b, :, :, o], ref, atol=1e-12)


def test_conv3x3_grad_input_is_the_transpose():
    rng = _rng(2)
    x = rng.normal(size=(2, 6, 5, 3))
    g = rng.normal(size=(2, 6, 5, 4))
    w = rng.normal(size=(9, 4, 3))
    lhs = np.sum(R.conv3x3(x, w) * g)
    rhs = np.sum(x * R.conv3x3_grad_input(g, w))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_conv3x3_grad_weight_by_linearity():
    # sum(g * conv(x, w)) is linear in w, so it equals <grad_weight(x, g), w>
    rng = _rng(3)
    x = rng.normal(size=(2, 5, 6, 3))
    g = rng.normal(size=(2, 5, 6, 4))
    for _ in range(3):
        w = rng.normal(size=(9, 4, 3))
        lhs = np.sum(g * R.conv3x3(x, w))
        rhs = np.sum(R.conv3x3_grad_weight(x, g) * w)
        assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_conv3x3_single_tap_is_a_shift():
    # a weight with one nonzero tap (ky, kx) shifts the image by (ky-1, kx-1)
    rng = _rng(4)
    x = rng.normal(size=(1, 5, 5, 1))
    for ky in range(3):
        for kx in range(3):
            w = np.zeros((9, 1, 1))
            w[3 * ky + kx, 0, 0] = 1.0
            y = R.conv3x3(x, w)[0, :, :, 0]
            for h in range(5):
                for c in range(5):
                    hh, cc = h + ky - 1, c + kx - 1
                    want = x[0, hh, cc, 0] if 0 <= hh < 5 and 0 <= cc < 5 else 0.0
                    assert y[h, c] == want


def test_pool_and_upsample_transposes():
    rng = _rng(5)
    a = rng.normal(size=(2, 8, 6, 3))
    c = rng.normal(size=(2, 4, 3, 3))
    assert abs(np.sum(R.avgpool2(a) * c) - np.sum(a * R.avgpool2_T(c))) < 1e-12
    assert abs(np.sum(R.upsample2(c) * a) - np.sum(c * R.upsample2_T(a))) < 1e-12
    assert np.allclose(R.avgpool2(R.upsample2(c)), c)
    assert np.allclose(R.avgpool2(np.full((1, 4, 4, 1), 2.5)), 2.5)


# ----------------------------------------------------------------------- U-Net
@pytest.mark.parametrize("levels,base", [(2, 2), (3, 2)])
def test_unet_gradient_matches_central_differences(levels, base):
    rng = _rng(6 + levels)
    shapes = [s for _, s in R.unet_layout(levels, base)]
    n = sum(int(np.prod(s)) for s in shapes)
    flat = rng.normal(size=n) * 0.5
    r = rng.normal(size=(2, 8, 8))
    e = rng.normal(size=(2, 8, 8))
    loss, g = R.precond_loss(flat, r, e, levels, base)
    h = 1e-6
    idx = rng.choice(n, 40, replace=False)
    for k in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        fd = (R.precond_loss(fp, r, e, levels, base)[0] - R.precond_loss(fm, r, e, levels, base)[0]) / (2 * h)
        assert abs(g[k] - fd) < 1e-6 * max(1.0, abs(fd)), (k, g[k], fd)


def test_unet_layout_counts():
    # 4 levels, 32 base channels: the parameter count written out by hand
    ch = [32, 64, 128, 256]
    n = 9 * (1 * 32 + 32 * 32)
    n += 9 * (32 * 64 + 64 * 64) + 9 * (64 * 128 + 128 * 128) + 9 * (128 * 256 + 256 * 256)
    for l in (2, 1, 0):
        n += 9 * (ch[l + 1] * ch[l] + 2 * ch[l] * ch[l] + ch[l] * ch[l])
    n += 32
    assert sum(int(np.prod(s)) for _, s in R.unet_layout(4, 32)) == n


def test_preconditioner_is_positively_homogeneous():
    # no biases and ReLU activations: N(a r) = a N(r) for a > 0, and the
    # input normalisation makes N exactly invariant in that sense
    rng = _rng(9)
    shapes = [s for _, s in R.unet_layout(3, 2)]
    flat = rng.normal(size=sum(int(np.prod(s)) for s in shapes))
    r = rng.normal(size=(1, 8, 8))
    z1 = R.precondition(flat, r, 3, 2)
    z2 = R.precondition(flat, 7.5 * r, 3, 2)
    assert np.allclose(z2, 7.5 * z1, rtol=1e-12, atol=1e-12)
    y, _ = R.unet_forward(flat, 3.0 * r, 3, 2)
    y1, _ = R.unet_forward(flat, r, 3, 2)
    assert np.allclose(y, 3.0 * y1, rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    # with bias correction the first step is lr * g / (|g| + eps): a sign step
    rng = _rng(10)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = R.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    assert np.allclose(p1 - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# --------------------------------------------------------- regulariser, solver
def test_regulariser_quadratic_form_and_null_space():
    rng = _rng(11)
    c = rng.normal(size=(7, 9))
    q = np.sum(c * R.reg_apply(c, 1.0))
    ref = np.sum(np.diff(c, axis=0) ** 2) + np.sum(np.diff(c, axis=1) ** 2)
    assert abs(q - ref) < 1e-10 * ref
    assert np.allclose(R.reg_apply(np.full((5, 6), 3.0), 2.0), 0.0)
    d = rng.normal(size=(7, 9))
    assert abs(np.sum(d * R.reg_apply(c, 1.0)) - np.sum(c * R.reg_apply(d, 1.0))) < 1e-10


def test_regulariser_neumann_eigenpairs():
    # the 1-D Neumann difference Laplacian has the DCT-II vectors as eigenvectors,
    # eigenvalue 4 sin^2(pi k / (2N)); the 2-D operator adds the two axes
    ny, nx = 6, 8
    j = np.arange(ny)[:, None] + 0.5
    i = np.arange(nx)[None, :] + 0.5
    for ky, kx in [(0, 1), (2, 0), (3, 5), (5, 7)]:
        v = np.cos(math.pi * ky * j / ny) * np.cos(math.pi * kx * i / nx)
        lam = 4 * math.sin(math.pi * ky / (2 * ny)) ** 2 + 4 * math.sin(math.pi * kx / (2 * nx)) ** 2
        assert np.allclose(R.reg_apply(v, 0.3), 0.3 * lam * v, atol=1e-12)


def _tiny_problem(n=1, N=6, seed=12):
    rng = _rng(seed)
    th = rng.uniform(0, math.pi, 14).astype(np.float32)
    y = rng.uniform(-3, 3, 14).astype(np.float32)
    lc = oracle.lines_from_theta_y(th, y)
    H = np.stack([oracle.forward(n, np.eye(N * N)[k].reshape(N, N), lc) for k in range(N * N)], axis=1)
    return lc, H


def test_normal_operator_matches_dense_matrix():
    n, N, lam = 1, 6, 0.05
    lc, H = _tiny_problem(n, N)
    Lt = np.stack([R.reg_apply(np.eye(N * N)[k].reshape(N, N), 1.0).ravel() for k in range(N * N)], axis=1)
    Mdense = H.T @ H + lam * Lt
    assert np.allclose(Mdense, Mdense.T, atol=1e-10)
    assert np.min(np.linalg.eigvalsh(Mdense)) > 0
    c = _rng(13).normal(size=(N, N))
    assert np.allclose(R.normal_apply(n, c, lc, lam).ravel(), Mdense @ c.ravel(), atol=1e-9)


def test_cg_solves_the_dense_system():
    n, N, lam = 1, 6, 0.05
    lc, H = _tiny_problem(n, N)
    b = _rng(14).normal(size=(N, N))
    x, it, hist = R.cg(lambda v: R.normal_apply(n, v, lc, lam), b, tol=1e-12, maxit=500)
    Lt = np.stack([R.reg_apply(np.eye(N * N)[k].reshape(N, N), 1.0).ravel() for k in range(N * N)], axis=1)
    xd = np.linalg.solve(H.T @ H + lam * Lt, b.ravel())
    assert np.allclose(x.ravel(), xd, rtol=1e-8, atol=1e-8)
    assert hist[-1] <= 1e-12 and it <= N * N + 20


def test_residual_loss_gradient_matches_central_differences():
    # the residual-space loss chains the network with the normal operator
    n, N, lam, levels, base = 1, 8, 0.05, 2, 2
    rng = _rng(15)
    th = rng.uniform(0, math.pi, 10).astype(np.float32)
    y = rng.uniform(-4, 4, 10).astype(np.float32)
    lc = oracle.lines_from_theta_y(th, y)
    shapes = [s for _, s in R.unet_layout(levels, base)]
    nprm = sum(int(np.prod(s)) for s in shapes)
    flat = rng.normal(size=nprm) * 0.5
    r = rng.normal(size=(2, N, N))
    loss, g = R.precond_loss_normal(flat, r, levels, base, n, lc, lam, gain=0.3)
    h = 1e-6
    for k in rng.choice(nprm, 25, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        fd = (R.precond_loss_normal(fp, r, levels, base, n, lc, lam, 0.3)[0]
              - R.precond_loss_normal(fm, r, levels, base, n, lc, lam, 0.3)[0]) / (2 * h)
        assert abs(g[k] - fd) < 1e-6 * max(1.0, abs(fd)), (k, g[k], fd)
    # the loss is the relative residual of one step x += N(r)
    z = R.precondition(flat, r, levels, base, gain=0.3)
    ref = np.mean([np.sum((R.normal_apply(n, z[b], lc, lam) - r[b]) ** 2) / np.sum(r[b] ** 2) for b in range(2)])
    assert abs(loss - ref) < 1e-12 * ref


@pytest.mark.parametrize("relu", [True, False])
def test_energy_loss_gradient_matches_central_differences(relu):
    # the energy-norm loss chains the network with the normal operator once
    n, N, lam, levels, base = 1, 8, 0.05, 2, 2
    rng = _rng(16)
    th = rng.uniform(0, math.pi, 10).astype(np.float32)
    y = rng.uniform(-4, 4, 10).astype(np.float32)
    lc = oracle.lines_from_theta_y(th, y)
    shapes = [s for _, s in R.unet_layout(levels, base)]
    nprm = sum(int(np.prod(s)) for s in shapes)
    flat = rng.normal(size=nprm) * 0.5
    e = rng.normal(size=(2, N, N))
    r = np.stack([R.normal_apply(n, e[b], lc, lam) for b in range(2)])
    loss, g = R.precond_loss_energy(flat, r, e, levels, base, n, lc, lam, gain=0.3, relu=relu)
    h = 1e-6
    for k in rng.choice(nprm, 25, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        fd = (R.precond_loss_energy(fp, r, e, levels, base, n, lc, lam, 0.3, relu)[0]
              - R.precond_loss_energy(fm, r, e, levels, base, n, lc, lam, 0.3, relu)[0]) / (2 * h)
        assert abs(g[k] - fd) < 1e-6 * max(1.0, abs(fd)), (k, g[k], fd)


def test_energy_loss_is_the_m_norm_of_the_step_error():
    # by the dense matrix M = H^T H + lam L^T L: loss = mean (z-e)^T M (z-e) / e^T M e
    # for pairs r = M e, z = N(r); an exact inverse (z = e) gives 0, z = 0 gives 1
    n, N, lam, levels, base = 1, 6, 0.05, 2, 2
    lc, H = _tiny_problem(n, N)
    Lt = np.stack([R.reg_apply(np.eye(N * N)[k].reshape(N, N), 1.0).ravel() for k in range(N * N)], axis=1)
    Md = H.T @ H + lam * Lt
    rng = _rng(17)
    shapes = [s for _, s in R.unet_layout(levels, base)]
    flat = rng.normal(size=sum(int(np.prod(s)) for s in shapes)) * 0.5
    e = rng.normal(size=(3, N, N))
    r = np.stack([(Md @ e[b].ravel()).reshape(N, N) for b in range(3)])
    for relu in (True, False):
        loss, _ = R.precond_loss_energy(flat, r, e, levels, base, n, lc, lam, gain=0.7, relu=relu)
        z = R.precondition(flat, r, levels, base, gain=0.7, relu=relu)
        ref = np.mean([(z[b] - e[b]).ravel() @ Md @ (z[b] - e[b]).ravel() / (e[b].ravel() @ Md @ e[b].ravel())
                       for b in range(3)])
        assert abs(loss - ref) < 1e-10 * ref
    # the out layer set to zero: N = 0, the step leaves the whole error
    flat0 = flat.copy()
    flat0[-base:] = 0.0
    loss0, _ = R.precond_loss_energy(flat0, r, e, levels, base, n, lc, lam, gain=0.7, relu=False)
    assert abs(loss0 - 1.0) < 1e-12


def test_linear_unet_is_a_linear_map():
    # without activations every layer is linear and there are no biases, so
    # N(a r1 + b r2) = a N(r1) + b N(r2) (the rms normalisation cancels);
    # with ReLU it is not
    rng = _rng(18)
    shapes = [s for _, s in R.unet_layout(3, 2)]
    flat = rng.normal(size=sum(int(np.prod(s)) for s in shapes))
    r1, r2 = rng.normal(size=(1, 8, 8)), rng.normal(size=(1, 8, 8))
    lin = R.precondition(flat, 2.0 * r1 - 3.0 * r2, 3, 2, relu=False)
    assert np.allclose(lin, 2.0 * R.precondition(flat, r1, 3, 2, relu=False)
                       - 3.0 * R.precondition(flat, r2, 3, 2, relu=False), rtol=1e-10, atol=1e-10)
    nl = R.precondition(flat, 2.0 * r1 - 3.0 * r2, 3, 2)
    assert not np.allclose(nl, 2.0 * R.precondition(flat, r1, 3, 2) - 3.0 * R.precondition(flat, r2, 3, 2),
                           rtol=1e-3, atol=1e-3)


# ------------------------------------------------- sinogram filter preconditioner
def test_sino_filter_matches_scipy_correlate1d():
    from scipy.ndimage import correlate1d
    rng = _rng(31)
    for n_views, n_bins, K in ((3, 17, 5), (2, 4, 9), (4, 40, 1), (1, 3, 63)):
        s = rng.normal(size=(n_views, n_bins))
        f = rng.normal(size=K)
        ref = correlate1d(s, f, axis=1, mode="constant", cval=0.0)
        got = R.sino_filter(s.ravel(), n_views, n_bins, f).reshape(n_views, n_bins)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_pcg_with_identity_is_cg_and_with_the_inverse_takes_one_step():
    n, N, lam = 1, 6, 0.05
    lc, H = _tiny_problem(n, N)
    b = _rng(32).normal(size=(N, N))
    A = lambda v: R.normal_apply(n, v, lc, lam)
    x1, it1, h1 = R.cg(A, b, tol=1e-10, maxit=200)
    x2, it2, h2 = R.pcg(A, lambda r: r, b, tol=1e-10, maxit=200)
    assert it1 == it2 and np.allclose(h1, h2, rtol=1e-9) and np.allclose(x1, x2, rtol=1e-9, atol=1e-12)
    Lt = np.stack([R.reg_apply(np.eye(N * N)[k].reshape(N, N), 1.0).ravel() for k in range(N * N)], axis=1)
    Minv = np.linalg.inv(H.T @ H + lam * Lt)
    x3, it3, _ = R.pcg(A, lambda r: (Minv @ r.ravel()).reshape(N, N), b, tol=1e-10, maxit=200)
    assert it3 == 1 and np.allclose(x3.ravel(), Minv @ b.ravel(), rtol=1e-9, atol=1e-12)


def test_sino_preconditioner_is_the_filtered_normal_product():
    # P r = H^T F H r + mu r with F the dense filter matrix of each view
    n, N = 1, 6
    lc, H = _tiny_problem(n, N)
    m = H.shape[0]
    n_views, n_bins = 1, m
    f = np.array([-1.0, 2.0, -1.0])
    F = np.stack([R.sino_filter(np.eye(m)[k], n_views, n_bins, f) for k in range(m)], axis=1)
    r = _rng(33).normal(size=(N, N))
    got = R.sino_precondition(n, r, lc, f, 0.25, n_views, n_bins)
    ref = (H.T @ (F @ (H @ r.ravel()))).reshape(N, N) + 0.25 * r
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)
    # a positive second difference filter gives a positive semi-definite P
    Pd = np.stack([R.sino_precondition(n, np.eye(N * N)[k].reshape(N, N), lc, f, 0.0, n_views, n_bins).ravel()
                   for k in range(N * N)], axis=1)
    assert np.allclose(Pd, Pd.T, atol=1e-10) and np.linalg.eigvalsh(0.5 * (Pd + Pd.T)).min() > -1e-10

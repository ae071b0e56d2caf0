"""FP64 CPU reference for the regularised reconstruction and its learned
preconditioner.

TEST INFRASTRUCTURE ONLY.  Like the rest of ``oracle/``, this module may be
imported only by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py``; it shares no code with ``paper_2503_20907_amd`` and the
GPU path never imports it.  Everything here is plain NumPy in float64, written
for a reader to check by eye; speed is not a goal.

What it computes:

* The inverse problem of Section IV-A (eq. (opti)): maximum-likelihood data
  term plus ``lambda R(c)``.  Reading used throughout: ``R(c) = 1/2 ||L c||^2``
  (Tikhonov) with ``L`` the forward differences along both grid axes and a
  Neumann boundary (no difference across the edge), so the minimiser solves
  the normal equations ``(H^T H + lambda L^T L) c = H^T p``.
* Conjugate gradients (Hestenes-Stiefel), the solver the paper runs on this
  problem (Section IV-B), and its preconditioned form with the sinogram-domain
  filter preconditioner ``P r = H^T (f * (H r)) + mu r`` (not in the paper).
* A small U-Net acting on a residual image (the learned preconditioner), its
  loss and its exact gradient by explicit back-propagation, and one Adam step
  (Kingma and Ba, 2015).  None of this is in the paper; the architecture is
  fixed in ``unet_layout`` and mirrored by the GPU library.

Array conventions: images are ``[ny][nx]`` (row ``j`` along x2, column ``i``
along x1); feature maps are NHWC ``[B][H][W][C]``; a 3x3 convolution weight is
``w[tap][c_out][c_in]`` with ``tap = 3*ky + kx`` reading input pixel
``(h + ky - 1, w + kx - 1)`` (zero outside the image).
"""
from __future__ import annotations

import numpy as np

from . import adjoint as _adjoint
from . import forward as _forward

# ---------------------------------------------------------------------------
# Regulariser and normal operator (Section IV-A, eq. (opti), Tikhonov reading)
# ---------------------------------------------------------------------------


def reg_apply(c, lam):
    """lam * L^T L c for forward differences with a Neumann boundary.

    (L_x c)[j, i] = c[j, i+1] - c[j, i] for i < nx-1 (none across the edge),
    and L_y likewise along rows.  L^T of a difference puts +d on the left
    point and -d on the right one, so the result at a pixel is
    (its value minus each in-grid neighbour), summed over those neighbours.
    """
    c = np.asarray(c, dtype=np.float64)
    out = np.zeros_like(c)
    dx = c[:, 1:] - c[:, :-1]          # L_x c
    out[:, :-1] -= dx                  # L_x^T: -d at the left point
    out[:, 1:] += dx                   #        +d at the right point
    dy = c[1:, :] - c[:-1, :]
    out[:-1, :] -= dy
    out[1:, :] += dy
    return lam * out


def normal_apply(n, c, line_cs, lam, spacing=1.0, cx=0.0, cy=0.0):
    """(H^T H + lam L^T L) c with the oracle's forward and adjoint."""
    c = np.asarray(c, dtype=np.float64)
    ny, nx = c.shape
    s = _forward(n, c, line_cs, spacing, cx, cy)
    return _adjoint(n, s, line_cs, nx, ny, spacing, cx, cy) + reg_apply(c, lam)


def cg(apply, b, tol=1e-3, maxit=1000, x0=None):
    """Conjugate gradients on an SPD operator (Hestenes-Stiefel).

    Stops when ||b - A x|| <= tol ||b|| with the recursively updated residual.
    Returns (x, iterations, list of relative residual norms).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    p = r.copy()
    rr = float(np.vdot(r, r))
    bn = float(np.sqrt(np.vdot(b, b)))
    hist = [np.sqrt(rr) / bn]
    it = 0
    while hist[-1] > tol and it < maxit:
        q = apply(p)
        alpha = rr / float(np.vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr) / bn)
    return x, it, hist


def pcg(apply, precond, b, tol=1e-3, maxit=1000):
    """Preconditioned conjugate gradients (Hestenes-Stiefel with z = P r) on an
    SPD operator with an SPD (or semi-definite) preconditioner ``precond``.

    Stops when ||b - A x|| <= tol ||b|| with the recursively updated residual.
    Returns (x, iterations, list of relative residual norms).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    bn = float(np.sqrt(np.vdot(b, b)))
    hist = [1.0]
    it = 0
    while hist[-1] > tol and it < maxit:
        q = apply(p)
        alpha = rz / float(np.vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        z = precond(r)
        rz_new = float(np.vdot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        hist.append(float(np.sqrt(np.vdot(r, r))) / bn)
    return x, it, hist


def sino_filter(s, n_views, n_bins, f):
    """out[v][j] = sum_k f[k] s[v][j + k - K//2] along each of the n_views
    runs of n_bins samples, zero outside a run (K = len(f) odd)."""
    s = np.asarray(s, dtype=np.float64).reshape(n_views, n_bins)
    f = np.asarray(f, dtype=np.float64)
    h = len(f) // 2
    out = np.zeros_like(s)
    for v in range(n_views):
        for j in range(n_bins):
            acc = 0.0
            for k in range(len(f)):
                jj = j + k - h
                if 0 <= jj < n_bins:
                    acc += f[k] * s[v, jj]
            out[v, j] = acc
    return out.ravel()


def sino_precondition(n, r, line_cs, f, mu, n_views, n_bins, spacing=1.0, cx=0.0, cy=0.0):
    """P r = H^T (f * (H r)) + mu r with the oracle's forward and adjoint."""
    r = np.asarray(r, dtype=np.float64)
    ny, nx = r.shape
    s = sino_filter(_forward(n, r, line_cs, spacing, cx, cy), n_views, n_bins, f)
    return _adjoint(n, s, line_cs, nx, ny, spacing, cx, cy) + mu * r


# ---------------------------------------------------------------------------
# U-Net building blocks, NHWC, float64
# ---------------------------------------------------------------------------


def _pad1(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))


def conv3x3(x, w):
    """y[b,h,w,o] = sum_{ky,kx,i} x[b,h+ky-1,w+kx-1,i] w[3ky+kx,o,i], zero padding."""
    x = np.asarray(x, dtype=np.float64)
    B, H, W, _ = x.shape
    xp = _pad1(x)
    y = np.zeros((B, H, W, w.shape[1]))
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + H, kx:kx + W, :] @ np.asarray(w[3 * ky + kx], np.float64).T
    return y


def conv3x3_grad_input(gy, w):
    """d/dx of sum(gy * conv3x3(x, w)): the transpose of the convolution."""
    gy = np.asarray(gy, dtype=np.float64)
    B, H, W, _ = gy.shape
    gp = _pad1(gy)
    gx = np.zeros((B, H, W, w.shape[2]))
    for ky in range(3):
        for kx in range(3):
            # x[h'] is read by output h = h' - ky + 1, i.e. padded index h' + 2 - ky
            gx += gp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W, :] @ np.asarray(w[3 * ky + kx], np.float64)
    return gx


def conv3x3_grad_weight(x, gy):
    """d/dw of sum(gy * conv3x3(x, w)), shape [9][c_out][c_in]."""
    x = np.asarray(x, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    B, H, W, ci = x.shape
    co = gy.shape[3]
    xp = _pad1(x)
    g2 = gy.reshape(-1, co)
    gw = np.zeros((9, co, ci))
    for ky in range(3):
        for kx in range(3):
            gw[3 * ky + kx] = g2.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, ci)
    return gw


def avgpool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_T(g):
    """Transpose of avgpool2: every fine pixel receives a quarter of its coarse value."""
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    """Nearest-neighbour 2x upsampling."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_T(g):
    B, H, W, C = g.shape
    return g.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ---------------------------------------------------------------------------
# The U-Net: layout, forward, loss, backward
# ---------------------------------------------------------------------------


def unet_layout(levels, base, max_channels=None):
    if isinstance(base, tuple):
        base, max_channels = base
    """Ordered list of (name, shape) of every parameter; the flat parameter
    vector is their concatenation in this order (row-major within each).

    Level l has c_l = base * 2^l channels, capped at max_channels if given.  Encoder level l: conv a
    (input -> c_l; the input is the 1-channel residual at l = 0, the 2x2
    average pool of level l-1's output otherwise), conv b (c_l -> c_l).
    Decoder level l (from levels-2 down to 0): conv up (c_{l+1} -> c_l, at
    level l+1's resolution, followed by nearest 2x upsampling), conv a on the
    concatenation [encoder output of level l, upsampled] (2 c_l -> c_l),
    conv b (c_l -> c_l).  Every 3x3 convolution is followed by ReLU and has no
    bias.  Output: a 1x1 convolution c_0 -> 1 without activation.
    """
    ch = [min(base << l, max_channels or (base << l)) for l in range(levels)]
    out = []
    for l in range(levels):
        cin = 1 if l == 0 else ch[l - 1]
        out.append((f"enc{l}a", (9, ch[l], cin)))
        out.append((f"enc{l}b", (9, ch[l], ch[l])))
    for l in range(levels - 2, -1, -1):
        out.append((f"dec{l}up", (9, ch[l], ch[l + 1])))
        out.append((f"dec{l}a", (9, ch[l], 2 * ch[l])))
        out.append((f"dec{l}b", (9, ch[l], ch[l])))
    out.append(("out", (ch[0],)))
    return out


def unpack(flat, levels, base):
    flat = np.asarray(flat, dtype=np.float64)
    p, o = {}, 0
    for name, shape in unet_layout(levels, base):
        k = int(np.prod(shape))
        p[name] = flat[o:o + k].reshape(shape)
        o += k
    assert o == flat.size, (o, flat.size)
    return p


def pack(p, levels, base):
    return np.concatenate([np.asarray(p[name], np.float64).ravel()
                           for name, _ in unet_layout(levels, base)])


def _relu(a):
    return np.maximum(a, 0.0)


def _ident(a):
    return a


def unet_forward(flat, x, levels, base, relu=True):
    """Network output for a batch of images x [B][H][W] (no normalisation).
    relu=False: the same network without its activations (a linear map).

    Returns (y [B][H][W], cache of every intermediate needed by the backward).
    """
    act = _relu if relu else _ident
    p = unpack(flat, levels, base)
    a = np.asarray(x, dtype=np.float64)[..., None]
    cache = {"x": a}
    enc = []
    for l in range(levels):
        if l > 0:
            a = avgpool2(enc[-1])
        cache[f"in{l}"] = a
        h = act(conv3x3(a, p[f"enc{l}a"]))
        cache[f"enc{l}h"] = h
        e = act(conv3x3(h, p[f"enc{l}b"]))
        enc.append(e)
    cache["enc"] = enc
    d = enc[-1]
    for l in range(levels - 2, -1, -1):
        cache[f"dec{l}in"] = d
        uc = act(conv3x3(d, p[f"dec{l}up"]))
        cache[f"dec{l}uc"] = uc
        cat = np.concatenate([enc[l], upsample2(uc)], axis=3)
        cache[f"dec{l}cat"] = cat
        h = act(conv3x3(cat, p[f"dec{l}a"]))
        cache[f"dec{l}h"] = h
        d = act(conv3x3(h, p[f"dec{l}b"]))
        cache[f"dec{l}d"] = d
    cache["last"] = d
    y = d @ p["out"]
    return y, cache


def unet_backward(flat, cache, gy, levels, base, relu=True):
    """Gradient of sum(gy * y) with respect to the flat parameter vector.

    Walks the forward in reverse: the 1x1 output, the decoder from the finest
    level to the coarsest, then the encoder from the coarsest level to the
    finest.  An encoder output receives gradient from two consumers (the
    pooled input of the next level and the decoder's concatenation); both are
    summed before that level is processed.
    """
    p = unpack(flat, levels, base)
    # derivative of the activation at a stored output (1 everywhere without)
    act = (lambda a: a > 0) if relu else (lambda a: 1.0)
    g = {}
    gy = np.asarray(gy, dtype=np.float64)
    g["out"] = np.einsum("bhwc,bhw->c", cache["last"], gy)
    gd = gy[..., None] * p["out"]                 # gradient of decoder level 0's output
    enc = cache["enc"]
    genc = [np.zeros_like(e) for e in enc]
    for l in range(levels - 1):                   # decoder, fine to coarse
        gpre = gd * act(cache[f"dec{l}d"])
        g[f"dec{l}b"] = conv3x3_grad_weight(cache[f"dec{l}h"], gpre)
        gh = conv3x3_grad_input(gpre, p[f"dec{l}b"]) * act(cache[f"dec{l}h"])
        g[f"dec{l}a"] = conv3x3_grad_weight(cache[f"dec{l}cat"], gh)
        gcat = conv3x3_grad_input(gh, p[f"dec{l}a"])
        c = enc[l].shape[3]
        genc[l] += gcat[..., :c]
        guc = upsample2_T(gcat[..., c:]) * act(cache[f"dec{l}uc"])
        g[f"dec{l}up"] = conv3x3_grad_weight(cache[f"dec{l}in"], guc)
        gd = conv3x3_grad_input(guc, p[f"dec{l}up"])   # gradient of decoder level l+1's output
    genc[levels - 1] += gd                        # the coarsest "decoder output" is the encoder's
    for l in range(levels - 1, -1, -1):           # encoder, coarse to fine
        gpre = genc[l] * act(enc[l])
        g[f"enc{l}b"] = conv3x3_grad_weight(cache[f"enc{l}h"], gpre)
        gh = conv3x3_grad_input(gpre, p[f"enc{l}b"]) * act(cache[f"enc{l}h"])
        g[f"enc{l}a"] = conv3x3_grad_weight(cache[f"in{l}"], gh)
        if l > 0:
            genc[l - 1] += avgpool2_T(conv3x3_grad_input(gh, p[f"enc{l}a"]))
    return pack(g, levels, base)


def precondition(flat, r, levels, base, gain=1.0, relu=True):
    """The learned preconditioner z = N(r) for a batch r [B][H][W]:
    N(r) = gain * rms(r) * UNet(r / rms(r)) per image (rms over its pixels)."""
    r = np.asarray(r, dtype=np.float64)
    rms = np.sqrt(np.mean(r * r, axis=(1, 2)))
    y, _ = unet_forward(flat, r / rms[:, None, None], levels, base, relu)
    return gain * y * rms[:, None, None]


def precond_loss(flat, r, e, levels, base, gain=1.0):
    """Training loss for pairs (r = M e, e) and its gradient.

    loss = mean_b ||N(r_b) - e_b||^2 / ||e_b||^2.  With s = 1/rms(r_b) this is
    ||UNet(s r_b) - s e_b / gain||^2 / ||s e_b / gain||^2, which is how it is
    evaluated.  Returns (loss, gradient w.r.t. the flat parameters).
    """
    r = np.asarray(r, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    B = r.shape[0]
    s = 1.0 / np.sqrt(np.mean(r * r, axis=(1, 2)))
    y, cache = unet_forward(flat, r * s[:, None, None], levels, base)
    t = e * s[:, None, None] / gain
    tn = np.sum(t * t, axis=(1, 2))
    diff = y - t
    loss = float(np.mean(np.sum(diff * diff, axis=(1, 2)) / tn))
    gy = 2.0 * diff / (tn[:, None, None] * B)
    return loss, unet_backward(flat, cache, gy, levels, base)


def adam_step(param, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) at step t >= 1.
    Returns new (param, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def precond_loss_normal(flat, r, levels, base, n, line_cs, lam, gain=1.0, nx=None, ny=None):
    """Residual-space training loss for the normal equations and its gradient.

    loss = mean_b ||M N(r_b) - r_b||^2 / ||r_b||^2, M = H^T H + lam L^T L (the
    oracle's transform).  With d_b = M z_b - r_b and z_b = N(r_b), the
    gradient w.r.t. z_b is 2 M d_b / (B ||r_b||^2) (M is symmetric), and
    z_b = gain rms(r_b) UNet(r_b / rms(r_b)) carries it to the network output.
    """
    r = np.asarray(r, dtype=np.float64)
    B = r.shape[0]
    rms = np.sqrt(np.mean(r * r, axis=(1, 2)))
    y, cache = unet_forward(flat, r / rms[:, None, None], levels, base)
    z = gain * y * rms[:, None, None]
    gy = np.zeros_like(y)
    loss = 0.0
    for b in range(B):
        d = normal_apply(n, z[b], line_cs, lam) - r[b]
        rr = float(np.sum(r[b] * r[b]))
        loss += float(np.sum(d * d)) / rr / B
        gz = 2.0 * normal_apply(n, d, line_cs, lam) / (B * rr)
        gy[b] = gz * gain * rms[b]
    return loss, unet_backward(flat, cache, gy, levels, base)


def precond_loss_energy(flat, r, e, levels, base, n, line_cs, lam, gain=1.0, relu=True):
    """Energy-norm training loss for the normal equations and its gradient.

    For pairs r_b = M e_b (M = H^T H + lam L^T L, the oracle's transform):
    loss = mean_b (z_b - e_b)^T M (z_b - e_b) / e_b^T M e_b with z_b = N(r_b),
    the squared M-norm of the error one step x += N(r) leaves, relative to the
    error's (conjugate gradients minimise this norm).  Written out with
    q_b = M z_b: (z^T q - 2 z^T r + e^T r) / e^T r, whose gradient w.r.t. z_b
    is 2 (q_b - r_b) / (B e_b^T r_b) (M is symmetric); z_b = gain rms(r_b)
    UNet(r_b / rms(r_b)) carries it to the network output.
    """
    r = np.asarray(r, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    B = r.shape[0]
    rms = np.sqrt(np.mean(r * r, axis=(1, 2)))
    y, cache = unet_forward(flat, r / rms[:, None, None], levels, base, relu)
    z = gain * y * rms[:, None, None]
    gy = np.zeros_like(y)
    loss = 0.0
    for b in range(B):
        q = normal_apply(n, z[b], line_cs, lam)
        er = float(np.sum(e[b] * r[b]))
        loss += (float(np.sum(z[b] * q)) - 2.0 * float(np.sum(z[b] * r[b])) + er) / er / B
        gy[b] = 2.0 * (q - r[b]) / (B * er) * gain * rms[b]
    return loss, unet_backward(flat, cache, gy, levels, base, relu)

"""Seeded synthetic inputs: line geometries and ellipse phantoms.

This module only draws inputs.  It holds none of the operator's arithmetic
(no footprint, no projection), so that the FP64 oracle and the HIP library can
both be fed from it without sharing any part of the method.

Geometry conventions (the line of eq. (1): {t theta + y theta^perp},
theta = (cos t, sin t), theta^perp = (sin t, -cos t)):

* parallel beam: angles t_m = m*pi/n_angles (m < n_angles, endpoint of [0, pi)
  excluded), computed in FP64 and rounded once to float32; detector bins
  y_j = (j - (n_bins-1)/2) * delta, centred on the origin; angle-major order.
* fan beam: source s on a circle of radius R at beta_m = 2*pi*m/n_src; bins on
  an equiangular arc centred on the ray through the origin, fan angles
  gamma_j = (j - (n_bins-1)/2) * 2*gamma_max/n_bins with
  gamma_max = asin(R_fov/R), R_fov = sqrt(2)*N/2 + (degree+1)/2 (the fan
  covers the padded grid).  Lines are delivered as float32 endpoint pairs
  (source, source + 2R*direction), source-major.
* random lines: t ~ U[0, pi), y ~ U[-N/2, N/2].

Phantom: E ellipses with centres U[-24,24]^2, semi-axes U[3,20] each,
rotation U[0,pi), amplitude U[-0.5,1], every length scaled by N/64; the
coefficient at grid centre x_k is the sum of the amplitudes of the ellipses
that contain x_k (no prefilter); optional i.i.d. texture N(0, sigma^2) with
sigma = 0.1 (the N(0, 0.01) of the workload read as a variance).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def parallel_beam(n_angles: int, n_bins: int, delta: float = 1.0, angle_range: float = math.pi):
    m = np.arange(n_angles, dtype=np.float64)
    th = (m * (angle_range / n_angles)).astype(np.float32)
    j = np.arange(n_bins, dtype=np.float64)
    yb = ((j - 0.5 * (n_bins - 1)) * delta).astype(np.float32)
    theta = np.repeat(th, n_bins)
    y = np.tile(yb, n_angles)
    return {"kind": "theta_y", "theta": theta, "y": y}


def fan_half_angle(N: int, degree: int, radius: float) -> float:
    r_fov = math.sqrt(2.0) * N / 2.0 + (degree + 1) / 2.0
    return math.asin(min(1.0, r_fov / radius))


def fan_beam(n_src: int, n_bins: int, radius: float, N: int, degree: int):
    gmax = fan_half_angle(N, degree, radius)
    beta = 2.0 * math.pi * np.arange(n_src, dtype=np.float64) / n_src
    gam = (np.arange(n_bins, dtype=np.float64) - 0.5 * (n_bins - 1)) * (2.0 * gmax / n_bins)
    sx = radius * np.cos(beta)
    sy = radius * np.sin(beta)
    # central direction points from the source to the origin
    phi = beta[:, None] + math.pi + gam[None, :]
    dx = np.cos(phi)
    dy = np.sin(phi)
    ep = np.empty((n_src, n_bins, 4), dtype=np.float64)
    ep[..., 0] = sx[:, None]
    ep[..., 1] = sy[:, None]
    ep[..., 2] = sx[:, None] + 2.0 * radius * dx
    ep[..., 3] = sy[:, None] + 2.0 * radius * dy
    return {"kind": "endpoints", "endpoints": ep.reshape(-1, 4).astype(np.float32)}


def random_lines(m: int, N: int, seed: int):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, math.pi, size=m).astype(np.float32)
    y = rng.uniform(-N / 2.0, N / 2.0, size=m).astype(np.float32)
    return {"kind": "theta_y", "theta": theta, "y": y}


def ellipse_phantom(N: int, n_ellipses: int, seed: int, texture_sigma: float = 0.0,
                    nx: int | None = None, ny: int | None = None):
    nx = N if nx is None else nx
    ny = N if ny is None else ny
    rng = np.random.default_rng(seed)
    sc = N / 64.0
    cen = rng.uniform(-24.0, 24.0, size=(n_ellipses, 2)) * sc
    ax = rng.uniform(3.0, 20.0, size=(n_ellipses, 2)) * sc
    rot = rng.uniform(0.0, math.pi, size=n_ellipses)
    amp = rng.uniform(-0.5, 1.0, size=n_ellipses)
    x1 = np.arange(nx, dtype=np.float64) - 0.5 * (nx - 1)
    x2 = np.arange(ny, dtype=np.float64) - 0.5 * (ny - 1)
    X1, X2 = np.meshgrid(x1, x2)  # [ny, nx]
    img = np.zeros((ny, nx), dtype=np.float64)
    for e in range(n_ellipses):
        c, s = math.cos(rot[e]), math.sin(rot[e])
        d1 = X1 - cen[e, 0]
        d2 = X2 - cen[e, 1]
        p = (c * d1 + s * d2) / ax[e, 0]
        q = (-s * d1 + c * d2) / ax[e, 1]
        img[p * p + q * q <= 1.0] += amp[e]
    if texture_sigma > 0.0:
        img += rng.normal(0.0, texture_sigma, size=img.shape)
    return img.astype(np.float32)


def concat_lines(*specs):
    """Concatenate line sets into one endpoint list (theta/y lines are turned
    into endpoint pairs at distance +-L along the line)."""
    eps = []
    for sp in specs:
        if sp["kind"] == "endpoints":
            eps.append(np.asarray(sp["endpoints"], dtype=np.float32))
        else:
            raise ValueError("concat_lines takes endpoint sets only")
    return {"kind": "endpoints", "endpoints": np.concatenate(eps, axis=0)}


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    N: int
    degree: int
    seed: int
    description: str


# Workloads (seeds fixed; recorded with every result)
SMALL_PARALLEL = Workload("parallel-64-deg1", 64, 1, 1,
                          "64x64 degree-1, parallel beam 90 angles x 96 bins, 10-ellipse phantom")
MEDIUM = Workload("mixed-512", 512, 3, 2,
                  "512x512 degrees 0-3, parallel 360x768 + fan 360x768 (R=1000), "
                  "30 ellipses + texture")
LARGE = Workload("fan+random-2048-cubic", 2048, 3, 5,
                 "2048x2048 cubic, fan 1440x3072 (R=4000) + 4,423,680 random lines")


def small_parallel():
    """64x64 degree-1 grid; 90 angles in [0, pi) x 96 bins of spacing 1."""
    w = SMALL_PARALLEL
    coeffs = ellipse_phantom(64, 10, seed=w.seed)
    return coeffs, parallel_beam(90, 96, 1.0)


def medium_parallel():
    w = MEDIUM
    coeffs = ellipse_phantom(512, 30, seed=w.seed, texture_sigma=0.1)
    return coeffs, parallel_beam(360, 768, 1.0)


def medium_fan(degree: int):
    w = MEDIUM
    coeffs = ellipse_phantom(512, 30, seed=w.seed, texture_sigma=0.1)
    return coeffs, fan_beam(360, 768, 1000.0, 512, degree)


def large_lines(n_src: int = 1440, n_bins: int = 3072, n_random: int | None = None,
                N: int = 2048, degree: int = 3, seed: int = 5):
    """Fan (R = 4000, same R/N as the 512 case) followed by random lines, as one
    endpoint list."""
    fan = fan_beam(n_src, n_bins, 4000.0, N, degree)
    nr = n_src * n_bins if n_random is None else n_random
    rnd = random_lines(nr, N, seed)
    th = rnd["theta"].astype(np.float64)
    y = rnd["y"].astype(np.float64)
    # a point on the line and a second point one radius along it
    px = y * np.sin(th)
    py = -y * np.cos(th)
    L = float(N)
    ep = np.stack([px - L * np.cos(th), py - L * np.sin(th),
                   px + L * np.cos(th), py + L * np.sin(th)], axis=1).astype(np.float32)
    return {"kind": "endpoints",
            "endpoints": np.concatenate([fan["endpoints"], ep], axis=0)}, fan["endpoints"].shape[0]


def large_phantom(N: int = 2048, seed: int = 5):
    return ellipse_phantom(N, 30, seed=seed, texture_sigma=0.1)


# ---------------------------------------------------------------------------
# Reconstruction inputs (regularised normal equations, learned preconditioner)
# ---------------------------------------------------------------------------


def recon_problem(N: int = 512, n_angles: int = 180, n_bins: int = 768, seed: int = 7):
    """Ground truth and geometry of the reconstruction workload: an N x N
    coefficient image (30 ellipses scaled by N/64 plus sigma = 0.1 texture)
    and parallel-beam lines, n_angles x n_bins at unit spacing."""
    return parallel_beam(n_angles, n_bins), ellipse_phantom(N, 30, seed, texture_sigma=0.1)


def noisy_log_data(clean, photons: float = 1e4, peak: float = 3.0, seed: int = 11):
    """Measured line integrals under Poisson noise: with kappa scaling the
    largest clean integral to `peak` attenuation, counts ~ Poisson(I0 exp(-kappa s)),
    counts of zero clamped to one, p = -ln(counts / I0) / kappa.  float32."""
    s = np.asarray(clean, dtype=np.float64)
    smax = float(np.max(np.abs(s)))
    kappa = peak / smax if smax > 0 else 1.0
    rng = np.random.default_rng(seed)
    counts = rng.poisson(photons * np.exp(-kappa * s)).astype(np.float64)
    counts = np.maximum(counts, 1.0)
    return (-np.log(counts / photons) / kappa).astype(np.float32)


def unet_params(shapes, seed: int):
    """He-normal draws (std sqrt(2/fan_in); a 1-D shape (an output layer) gets
    std sqrt(1/fan_in)) for a list of parameter shapes [taps][c_out][c_in] or
    [c_in], concatenated into one float32 vector."""
    rng = np.random.default_rng(seed)
    out = []
    for shape in shapes:
        if len(shape) == 1:
            sd = math.sqrt(1.0 / shape[0])
        else:
            sd = math.sqrt(2.0 / (shape[0] * shape[2]))
        out.append(rng.normal(0.0, sd, size=int(np.prod(shape))))
    return np.concatenate(out).astype(np.float32)


def training_fields(count: int, H: int, W: int, seed: int, device="cpu"):
    """`count` error images e for (M e, e) training pairs, float32 [count][H][W],
    each scaled to unit RMS.  Even indices: ellipse phantoms (5-30 ellipses,
    centres within the grid, semi-axes 2-35% of the size, amplitudes U[-1, 1]);
    odd indices: Gaussian random fields with power spectrum
    (|k|^2 + k0^2)^(-alpha), alpha ~ U[0, 2.5], k0 ~ U[0.005, 0.1] cycles per
    pixel (from white noise to smooth fields).  Drawn with torch on `device`."""
    import torch
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    out = torch.empty((count, H, W), dtype=torch.float32, device=dev)
    yy = (torch.arange(H, device=dev, dtype=torch.float32) - 0.5 * (H - 1))[:, None]
    xx = (torch.arange(W, device=dev, dtype=torch.float32) - 0.5 * (W - 1))[None, :]
    size = float(min(H, W))
    ky = torch.fft.fftfreq(H, device=dev)[:, None]
    kx = torch.fft.rfftfreq(W, device=dev)[None, :]
    k2 = ky * ky + kx * kx

    def u(*shape, lo=0.0, hi=1.0):
        return lo + (hi - lo) * torch.rand(*shape, generator=g, device=dev)

    for i in range(count):
        if i % 2 == 0:
            E = int(u(1, lo=5, hi=31).item())
            cx, cy = u(E, lo=-0.45, hi=0.45) * W, u(E, lo=-0.45, hi=0.45) * H
            a, b = u(E, lo=0.02, hi=0.35) * size, u(E, lo=0.02, hi=0.35) * size
            th = u(E, hi=math.pi)
            amp = u(E, lo=-1.0, hi=1.0)
            c, s = torch.cos(th)[:, None, None], torch.sin(th)[:, None, None]
            dx, dy = xx[None] - cx[:, None, None], yy[None] - cy[:, None, None]
            xr, yr = c * dx + s * dy, -s * dx + c * dy
            inside = (xr / a[:, None, None]) ** 2 + (yr / b[:, None, None]) ** 2 <= 1.0
            img = (inside.float() * amp[:, None, None]).sum(0)
        else:
            alpha = float(u(1, hi=2.5).item())
            k0 = float(u(1, lo=0.005, hi=0.1).item())
            noise = torch.randn((H, W), generator=g, device=dev)
            spec = torch.fft.rfft2(noise) * (k2 + k0 * k0) ** (-alpha / 2.0)
            img = torch.fft.irfft2(spec, s=(H, W))
        rms = torch.sqrt(torch.mean(img * img))
        out[i] = img / rms if float(rms) > 0 else img
    return out


# ---------------------------------------------------------------------------
# Batches of uneven problems
# ---------------------------------------------------------------------------


def batch_problems(count: int = 64, seed: int = 21, sizes=(128, 256, 512, 1024), degrees=(1, 3),
                   angles=(60, 720), phantoms: bool = True):
    """`count` problems of uneven size: N drawn from `sizes`, degree from
    `degrees`, the number of views U{angles}, parallel beam or fan beam with
    equal probability, ceil(1.5 N) unit-spaced bins (parallel) or bins on the
    arc (fan, source radius 2N).  Returns a list of dicts with N, degree,
    kind, spec (lines), and the phantom (30 ellipses + texture)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.choice(sizes))
        n = int(rng.choice(degrees))
        na = int(rng.integers(angles[0], angles[1] + 1))
        nb = int(math.ceil(1.5 * N))
        if rng.random() < 0.5:
            spec, kind = parallel_beam(na, nb), "parallel"
        else:
            spec, kind = fan_beam(na, nb, 2.0 * N, N, n), "fan"
        out.append({"N": N, "degree": n, "kind": kind, "views": na, "bins": nb, "spec": spec,
                    "phantom": ellipse_phantom(N, 30, seed * 1000 + i, texture_sigma=0.1) if phantoms else None})
    return out

"""Seeded synthetic workloads for the Kronecker-product SVD / split Bregman path.

This module only *draws* inputs: point-spread functions (PSFs), test images,
noise and Gaussian start blocks. It holds none of the method's arithmetic
(no rearrangement, no bidiagonalization, no sketching, no regularization).
Both the CPU oracle and the HIP path consume what it returns, so they always
see identical inputs.

Conventions (shared by every consumer):

* An n x n image ``X`` is a NumPy array indexed ``X[row, col]`` with ``row``
  the vertical coordinate. The paper's ``vec`` is column-major, so the vector
  form of ``X`` is ``X.flatten(order="F")`` (pixel (r, c) -> index r + n*c).
* A PSF is a 2-D array ``P[u, v]`` (u = vertical offset, v = horizontal
  offset) with centre ``(cu, cv)``. With zero boundary conditions the blurred
  image is ``B[r, i] = sum_{c,j} P[cu + r - c, cv + i - j] X[c, j]``, the
  forward model of the paper's introduction (eq. "forward problem").
* The configured PSFs live on the full offset grid of an n x n image:
  shape (2n-1, 2n-1), centre (n-1, n-1), unit sum.

The paper's own test problems (IR Tools speckle PSFs and images) are not
available, so these generators stand in for them; the recipe is stated with
each function.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.signal

# Seed bases for the synthetic workloads; config i adds i.
SEED_PSF = 1000
SEED_IMAGE = 2000
SEED_NOISE = 3000
SEED_START = 4000
SEED_ARRIVALS = 5000


def _offsets(n: int):
    """Vertical and horizontal offset grids of the full (2n-1)^2 PSF support."""
    d = np.arange(-(n - 1), n, dtype=np.float64)
    u, v = np.meshgrid(d, d, indexing="ij")
    return u, v


def gaussian_psf(n: int, sigmas=(2.0, 1.0), theta_deg: float = 30.0):
    """Rotated (non-separable) Gaussian on the full offset grid.

    P[u, v] ~ exp(-(x'^2/s1^2 + y'^2/s2^2)/2) with x' = v cos t + u sin t and
    y' = -v sin t + u cos t, normalized to unit sum. Returns (P, cu, cv).
    """
    u, v = _offsets(n)
    t = math.radians(theta_deg)
    xp = v * math.cos(t) + u * math.sin(t)
    yp = -v * math.sin(t) + u * math.cos(t)
    P = np.exp(-0.5 * ((xp / sigmas[0]) ** 2 + (yp / sigmas[1]) ** 2))
    P /= P.sum()
    return P, n - 1, n - 1


def disk_psf(n: int, radius: float = 8.0):
    """Defocus disk: 1/|D| on the pixel centres with u^2 + v^2 <= r^2."""
    u, v = _offsets(n)
    P = ((u * u + v * v) <= radius * radius).astype(np.float64)
    P /= P.sum()
    return P, n - 1, n - 1


def motion_psf(n: int, length: int = 15, theta: float | None = None,
               seed: int = SEED_PSF, samples_per_pixel: int = 20):
    """Straight motion blur of the given length (pixels) at angle theta (rad).

    The segment t in [-(L-1)/2, (L-1)/2] is sampled with ``samples_per_pixel``
    points per pixel of length and bilinearly splatted onto the grid. When
    theta is None it is drawn from U[0, pi) with ``seed``.
    """
    if theta is None:
        theta = float(np.random.default_rng(seed).uniform(0.0, math.pi))
    half = (length - 1) / 2.0
    ns = samples_per_pixel * length
    ts = np.linspace(-half, half, ns)
    uu = ts * math.sin(theta)          # vertical offset
    vv = ts * math.cos(theta)          # horizontal offset
    P = np.zeros((2 * n - 1, 2 * n - 1))
    c = n - 1
    u0 = np.floor(uu).astype(int)
    v0 = np.floor(vv).astype(int)
    fu = uu - u0
    fv = vv - v0
    for du, wu in ((0, 1.0 - fu), (1, fu)):
        for dv, wv in ((0, 1.0 - fv), (1, fv)):
            iu = u0 + du + c
            iv = v0 + dv + c
            ok = (iu >= 0) & (iu < 2 * n - 1) & (iv >= 0) & (iv < 2 * n - 1)
            np.add.at(P, (iu[ok], iv[ok]), (wu * wv)[ok])
    P /= P.sum()
    return P, c, c


def speckle_psf(n: int, seed: int = SEED_PSF, m: int = 64,
                pupil_diameter: float = 24.0, phase_rms: float = 6.0):
    """Speckle-like PSF, |FFT2(pupil * exp(i phi))|^2 (generic optics model).

    phi is white Gaussian noise filtered by |f|^(-11/6) and scaled to
    ``phase_rms`` radians RMS over the pupil. The m x m intensity pattern is
    centred on the offset grid (cropped if the grid is smaller) and normalized.
    """
    rng = np.random.default_rng(seed)
    fy = np.fft.fftfreq(m)[:, None]
    fx = np.fft.fftfreq(m)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    filt = f ** (-11.0 / 6.0)
    filt[0, 0] = 0.0
    noise = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    phi = np.real(np.fft.ifft2(noise * filt))
    yy, xx = np.meshgrid(np.arange(m) - m / 2 + 0.5, np.arange(m) - m / 2 + 0.5,
                         indexing="ij")
    pupil = (xx * xx + yy * yy) <= (pupil_diameter / 2.0) ** 2
    phi = phi - phi[pupil].mean()
    phi *= phase_rms / np.sqrt(np.mean(phi[pupil] ** 2))
    field = pupil * np.exp(1j * phi)
    inten = np.abs(np.fft.fftshift(np.fft.fft2(field))) ** 2
    P = np.zeros((2 * n - 1, 2 * n - 1))
    c = n - 1
    h = min(n - 1, m // 2 - 1)
    P[c - h:c + h + 1, c - h:c + h + 1] = inten[m // 2 - h:m // 2 + h + 1,
                                                m // 2 - h:m // 2 + h + 1]
    P /= P.sum()
    return P, c, c


def random_psf(pu: int, pv: int, seed: int, cu: int | None = None,
               cv: int | None = None):
    """Asymmetric, generally off-centre random PSF (test fixture)."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.0, 1.0, size=(pu, pv))
    P /= P.sum()
    if cu is None:
        cu = int(rng.integers(0, pu))
    if cv is None:
        cv = int(rng.integers(0, pv))
    return P, cu, cv


def separable_psf(a: np.ndarray, b: np.ndarray):
    """P = a b^T (rank-1 PSF); centre at the middle of each factor."""
    P = np.outer(a, b)
    return P, len(a) // 2, len(b) // 2


def rectangles_image(n: int, seed: int = SEED_IMAGE, count: int = 8):
    """Piecewise-constant test image: ``count`` random rectangles on zero.

    Side lengths ~ U[n/8, n/3], positions uniform, intensity ~ U[0.2, 1];
    later rectangles overwrite earlier ones.
    """
    rng = np.random.default_rng(seed)
    X = np.zeros((n, n))
    lo = max(1, n // 8)
    hi = max(lo + 1, n // 3)
    for _ in range(count):
        h = int(rng.integers(lo, hi + 1))
        w = int(rng.integers(lo, hi + 1))
        r0 = int(rng.integers(0, n - h + 1))
        c0 = int(rng.integers(0, n - w + 1))
        X[r0:r0 + h, c0:c0 + w] = rng.uniform(0.2, 1.0)
    return X


def blur_zero_bc(P: np.ndarray, cu: int, cv: int, X: np.ndarray) -> np.ndarray:
    """Forward model B = A X (zero boundary conditions) via full 2-D convolution.

    B[r, i] = sum_{c,j} P[cu + r - c, cv + i - j] X[c, j] is the window
    [cu : cu+n, cv : cv+n] of the full linear convolution of X with P (a direct
    sum for small sizes, an FP64 FFT convolution for large ones).
    """
    n = X.shape[0]
    if n * n * P.size <= (1 << 26):
        full = scipy.signal.convolve2d(X, P, mode="full")      # direct sum
    else:
        full = scipy.signal.fftconvolve(X, P, mode="full")     # FP64 FFT, large images
    return full[cu:cu + n, cv:cv + n].copy()


def add_noise(b_true: np.ndarray, level: float, seed: int = SEED_NOISE):
    """b = b_true + eta, eta = level * (||b_true|| / ||zeta||) * zeta, zeta ~ N(0, I).

    The scaling is the paper's noise model (section "Performance Metrics").
    """
    rng = np.random.default_rng(seed)
    zeta = rng.standard_normal(b_true.shape)
    eta = level * (np.linalg.norm(b_true) / np.linalg.norm(zeta)) * zeta
    return b_true + eta


def gaussian_block(rows: int, cols: int, seed: int = SEED_START) -> np.ndarray:
    """N(0, 1) block (start vector y when cols == 1, sketch F otherwise),
    column-major semantics: column t is ``out[:, t]``."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((rows, cols))


def deblur_problem(n: int, psf: str = "gaussian", noise: float = 0.01, idx: int = 0):
    """A full synthetic deblurring instance: (P, cu, cv, x_true, b_true, b)."""
    if psf == "gaussian":
        P, cu, cv = gaussian_psf(n)
    elif psf == "disk":
        P, cu, cv = disk_psf(n)
    elif psf == "motion":
        P, cu, cv = motion_psf(n, seed=SEED_PSF + idx)
    elif psf == "speckle":
        P, cu, cv = speckle_psf(n, seed=SEED_PSF + idx)
    else:
        raise ValueError(psf)
    x_true = rectangles_image(n, seed=SEED_IMAGE + idx)
    b_true = blur_zero_bc(P, cu, cv, x_true)
    b = add_noise(b_true, noise, seed=SEED_NOISE + idx)
    return P, cu, cv, x_true, b_true, b


# ---------------------------------------------------------------------------
# Mixed workloads: many problems of uneven size and PSF (batched KP-SVD) and a
# request stream with recurring PSFs (deblurring server).

FAMILIES = ("gaussian", "motion", "disk")


def mixed_psf(n: int, family: str, rng: np.random.Generator):
    """One PSF of the given family with randomly drawn shape parameters:
    Gaussian sigma1 ~ U[1, 3], sigma2 ~ U[0.5, sigma1], theta ~ U[0, 180) deg;
    motion length 15 at theta ~ U[0, pi); disk radius ~ U[3, 8]."""
    if family == "gaussian":
        s1 = float(rng.uniform(1.0, 3.0))
        s2 = float(rng.uniform(0.5, s1))
        return gaussian_psf(n, (s1, s2), float(rng.uniform(0.0, 180.0)))
    if family == "motion":
        return motion_psf(n, 15, float(rng.uniform(0.0, math.pi)))
    if family == "disk":
        return disk_psf(n, float(rng.uniform(3.0, 8.0)))
    raise ValueError(family)


def batched_mix(count: int = 64, sizes=(128, 192, 256, 384, 512), ranks=(10, 30),
                p: int = 10, seed: int = SEED_PSF + 500):
    """``count`` KP-SVD problems: n ~ U(sizes), family ~ U(FAMILIES),
    rank k ~ U{ranks[0] .. ranks[1]}, oversampling / enlargement p."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        fam = FAMILIES[int(rng.integers(0, len(FAMILIES)))]
        P, cu, cv = mixed_psf(n, fam, rng)
        k = int(rng.integers(ranks[0], ranks[1] + 1))
        out.append(dict(n=n, family=fam, P=P, cu=cu, cv=cv, k=k, p=p, seed=SEED_START + i))
    return out


def serving_psf(psf_id: int, n: int):
    """PSF number ``psf_id`` of the recurring set, on the offset grid of n:
    the family cycles through FAMILIES and the shape parameters are drawn from
    a generator seeded by the id, so a PSF is the same for every image size."""
    rng = np.random.default_rng(SEED_PSF + 700 + psf_id)
    return mixed_psf(n, FAMILIES[psf_id % len(FAMILIES)], rng)


def serving_stream(count: int = 2000, rate: float = 200.0, sizes=(128, 256, 512, 1024),
                   weights=(4, 3, 2, 1), n_psf: int = 16, seed: int = SEED_ARRIVALS):
    """Open-loop Poisson request stream: exponential inter-arrival times of
    mean 1/rate seconds, n drawn with the given weights, PSF id ~ U{0..n_psf-1},
    isotropic or anisotropic with probability 1/2 each."""
    rng = np.random.default_rng(seed)
    w = np.asarray(weights, dtype=np.float64)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    n = rng.choice(np.asarray(sizes), size=count, p=w / w.sum())
    psf = rng.integers(0, n_psf, size=count)
    iso = rng.integers(0, 2, size=count)
    return [dict(t=float(t[i]), n=int(n[i]), psf_id=int(psf[i]), iso=bool(iso[i]))
            for i in range(count)]

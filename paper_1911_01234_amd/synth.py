"""Seeded synthetic inputs for variable-density partial-Fourier MRI.

This module builds the *problem*, never the reconstruction: ellipse phantoms with a
smooth phase, Bernoulli variable-density sampling sets with their probabilities p_j,
and the noisy zero-filled measurements of the measurement model (Section 1, eq. 1:
y = Phi x0 + eps, Phi = M_Omega F, eps ~ CN(0, sigma^2 I) with white phase).  It holds
none of the method's arithmetic and is shared by the tests, the benchmark and the
CPU oracle's callers.

Stand-in for the paper's workload (Section 3: a 512x512 Shepp-Logan phantom, 40 dB,
polynomial variable density, undersampling about 4, 6 and 8): random-ellipse phantoms
replace the Shepp-Logan table (which is not reproduced here), and the density is the
polynomial (1 - r)^d raised by a constant offset, clipped to [0, 1], with a fully
sampled centre block; the offset is found by bisection so that sum(p) = N / R.

Conventions
-----------
* Images are complex, row-major ``[ny][nx]``; axis 0 is y, axis 1 is x.
* Grid coordinates u = 2 (j + 0.5) / n - 1 on both axes (x along columns).
* The unitary DFT is used for the measurements, natural (un-centred) k-space order.
* Random streams: ``SeedSequence([cfg_id, slice_id, stream])`` with
  stream 0 = phantom, 1 = phase, 2 = mask, 3 = noise, 4 = texture.
* SNR definition (Section 3): ||F x0||^2 / (N sigma^2) = 10^(SNR/10); with the unitary
  F this is sigma^2 = ||x0||^2 / (N 10^(SNR/10)).  E|eps_j|^2 = sigma^2, real and
  imaginary parts i.i.d. N(0, sigma^2 / 2).
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np

STREAM_PHANTOM, STREAM_PHASE, STREAM_MASK, STREAM_NOISE, STREAM_TEXTURE = range(5)


def rng_for(cfg_id: int, slice_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([int(cfg_id), int(slice_id), int(stream)])))


def _grid(ny: int, nx: int):
    v = 2.0 * (np.arange(ny) + 0.5) / ny - 1.0
    u = 2.0 * (np.arange(nx) + 0.5) / nx - 1.0
    return np.meshgrid(u, v)  # U varies along x (columns), V along y (rows)


def _paint_ellipses(U, V, rng, count, body, mag=None):
    """Painter's-order ellipses; returns the magnitude image and the list of masks."""
    if mag is None:
        mag = np.zeros(U.shape)
    masks = []
    for e in range(count):
        if body and e == 0:
            cx, cy = rng.uniform(-0.1, 0.1, size=2)
            a, b = rng.uniform(0.6, 0.85, size=2)
        else:
            cx, cy = rng.uniform(-0.5, 0.5, size=2)
            a, b = rng.uniform(0.05, 0.4, size=2)
        ang = rng.uniform(0.0, np.pi)
        inten = rng.uniform(0.1, 1.0)
        du, dv = U - cx, V - cy
        ca, sa = np.cos(ang), np.sin(ang)
        ur = ca * du + sa * dv
        vr = -sa * du + ca * dv
        inside = (ur / a) ** 2 + (vr / b) ** 2 <= 1.0
        mag[inside] = inten
        masks.append(inside)
    return mag, masks


def _texture_field(ny, nx, rng, sigma_px=2.0):
    """Gaussian white noise, periodically smoothed by a Gaussian of width sigma_px,
    standardised to zero mean and unit variance."""
    g = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    H = np.exp(-2.0 * (np.pi * sigma_px) ** 2 * (ky ** 2 + kx ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(g) * H))
    f -= f.mean()
    sd = f.std()
    return f / sd if sd > 0 else f


def phantom(cfg_id: int, slice_id: int, ny: int, nx: int, n_ellipses: int,
            texture: bool = False) -> np.ndarray:
    """Complex phantom x0 = magnitude * exp(i phi), complex128 [ny][nx]."""
    U, V = _grid(ny, nx)
    mag, _ = _paint_ellipses(U, V, rng_for(cfg_id, slice_id, STREAM_PHANTOM), n_ellipses, True)
    if texture:
        trng = rng_for(cfg_id, slice_id, STREAM_TEXTURE)
        G = _texture_field(ny, nx, trng)
        _, regions = _paint_ellipses(U, V, trng, 8, False, mag=np.zeros_like(mag))
        for m in regions:
            mag[m] = np.maximum(mag[m] * (1.0 + 0.25 * G[m]), 0.0)
    prng = rng_for(cfg_id, slice_id, STREAM_PHASE)
    c = prng.uniform(-1.0, 1.0, size=6)
    phi = (c[0] + c[1] * U + c[2] * V + c[3] * U * U + c[4] * U * V + c[5] * V * V)
    pm = np.abs(phi).max()
    if pm > 0:
        phi = phi * (np.pi / 4.0) / pm
    return mag * np.exp(1j * phi)


@functools.lru_cache(maxsize=64)
def _density_centred(ny: int, nx: int, R: float, d: float, C: int, scaling: str) -> np.ndarray:
    ky = np.arange(-(ny // 2), ny - ny // 2)[:, None].astype(np.float64)
    kx = np.arange(-(nx // 2), nx - nx // 2)[None, :].astype(np.float64)
    rad = np.sqrt(ky ** 2 + kx ** 2)
    r = rad / rad.max()
    base = (1.0 - r) ** d
    centre = (ky >= -(C // 2)) & (ky < C - C // 2) & (kx >= -(C // 2)) & (kx < C - C // 2)
    target = ny * nx / float(R)
    if target > ny * nx or target < centre.sum():
        raise ValueError("undersampling factor incompatible with the fully sampled centre")

    if scaling == "offset":
        def prob(c):
            return np.clip(base + c, 0.0, 1.0)
        lo, hi = -1.0, 1.0
    elif scaling == "multiplicative":
        def prob(c):
            return np.minimum(1.0, c * base)
        lo, hi = 0.0, 1.0
        while np.minimum(1.0, hi * base).sum() < target:
            hi *= 2.0
    else:
        raise ValueError(scaling)

    def total(c):
        p = prob(c)
        p[centre] = 1.0
        return p.sum()

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < target:
            lo = mid
        else:
            hi = mid
    p = prob(hi)
    p[centre] = 1.0
    p.setflags(write=False)
    return p


def density(ny: int, nx: int, R: float, d: float, C: int, scaling: str = "offset") -> np.ndarray:
    """Sampling probabilities p_j in natural FFT order (float64 [ny][nx]).

    Polynomial variable density in the normalised radius r = |k| / max|k| (centred
    coordinates, the corner has r = 1) with a fully sampled C x C centre block:
    * ``"offset"`` (default): p = clip((1 - r)^d + c, 0, 1), the offset c set by
      bisection so that sum(p) = N / R;
    * ``"multiplicative"``: p = min(1, c (1 - r)^d), c set the same way.  Here p falls
      to 0 toward the corner and density compensation (1/p) amplifies the measurement
      noise by up to 1/min(p); kept for comparison.
    """
    return np.fft.ifftshift(_density_centred(ny, nx, float(R), float(d), int(C), scaling))


@dataclass
class Slice:
    x0: np.ndarray       # complex128 [ny][nx] ground truth
    y: np.ndarray        # complex128 [ny][nx] zero-filled measurements, natural order
    mask: np.ndarray     # uint8 [ny][nx], 1 where j in Omega
    p: np.ndarray        # float64 [ny][nx], sampling probability
    sigma2: float        # E|eps_j|^2
    R: float
    snr_db: float


def make_slice(cfg_id: int, slice_id: int, ny: int, nx: int, n_ellipses: int, R: float,
               d: float, C: int, snr_db: float, texture: bool = False,
               scaling: str = "offset") -> Slice:
    x0 = phantom(cfg_id, slice_id, ny, nx, n_ellipses, texture)
    p = density(ny, nx, R, d, C, scaling)
    mrng = rng_for(cfg_id, slice_id, STREAM_MASK)
    mask = (mrng.random((ny, nx)) < p).astype(np.uint8)
    N = ny * nx
    sigma2 = float(np.sum(np.abs(x0) ** 2) / (N * 10.0 ** (snr_db / 10.0)))
    nrng = rng_for(cfg_id, slice_id, STREAM_NOISE)
    eps = (nrng.standard_normal((ny, nx)) + 1j * nrng.standard_normal((ny, nx))) * np.sqrt(sigma2 / 2.0)
    y = mask * (np.fft.fft2(x0, norm="ortho") + eps)
    return Slice(x0=x0, y=y, mask=mask, p=p, sigma2=sigma2, R=float(R), snr_db=float(snr_db))


# ---------------------------------------------------------------------------------
# Workload recipes.  Each returns a list of Slice objects plus the wavelet depth and
# the iteration count.

def workload_single64(slice_id: int = 0):
    """64x64, 8 ellipses, p ~ (1-r)^4, 8x8 centre, R=4, 30 dB, 3 Haar levels, 30 iterations."""
    return [make_slice(1, slice_id, 64, 64, 8, 4.0, 4.0, 8, 30.0)], 3, 30


def workload_single256(R: float = 4.0, slice_id: int = 0):
    """256x256, 16 ellipses, p ~ (1-r)^6, 16x16 centre, 40 dB, 4 Haar levels, 50 iterations."""
    return [make_slice(2, slice_id, 256, 256, 16, R, 6.0, 16, 40.0)], 4, 50


def workload_batch256(batch: int, cfg_id: int = 6, Rs=(4.0, 6.0, 8.0), first_slice: int = 0):
    """A batch of independent 256x256 slices of the single-256 recipe; slice b uses
    R = Rs[b % len(Rs)] and its own seeds."""
    out = []
    for b in range(first_slice, first_slice + batch):
        out.append(make_slice(cfg_id, b, 256, 256, 16, Rs[b % len(Rs)], 6.0, 16, 40.0))
    return out, 4, 50


def workload_mixed(n_per_size: int = 128, sizes=(128, 192, 256, 320), cfg_id: int = 3):
    """Mixed batch: n_per_size slices of each square size, order shuffled by seed;
    R ~ U{4,6,8,10}, SNR ~ U[25,45] dB, 16 ellipses, d=6, 16x16 centre, 4 levels, 50 iters."""
    total = n_per_size * len(sizes)
    rng = rng_for(cfg_id, 1 << 20, 0)
    order = rng.permutation(total)
    Rs = rng.choice([4.0, 6.0, 8.0, 10.0], size=total)
    snrs = rng.uniform(25.0, 45.0, size=total)
    out = []
    for i in range(total):
        n = sizes[order[i] % len(sizes)]
        out.append(make_slice(cfg_id, i, n, n, 16, Rs[i], 6.0, 16, snrs[i]))
    return out, 4, 50


def workload_batch512(batch: int, cfg_id: int = 5, Rs=(8.0, 12.0), first_slice: int = 0):
    """512x512 slices: 32 ellipses plus textured regions (filtered Gaussian noise),
    p ~ (1-r)^6 with a 16x16 centre, R cycling over Rs (8x and 12x), 40 dB, 4 Haar levels,
    50 iterations (the recipe of workload_c5)."""
    out = []
    for b in range(first_slice, first_slice + batch):
        out.append(make_slice(cfg_id, b, 512, 512, 32, Rs[b % len(Rs)], 6.0, 16, 40.0, texture=True))
    return out, 4, 50


def workload_c4(n: int, cfg_id: int = 40, first_slice: int = 0):
    """Slices for the learned denoiser at 256x256 (training cfg_id 40, evaluation 41,
    validation 42): the single-256 recipe (16 ellipses, p ~ (1-r)^6, 16x16 centre) with
    R ~ U{4, 6, 8} and SNR ~ U[30, 45] dB drawn per slice from the slice's own seeds;
    4 Haar levels, 50 iterations."""
    out = []
    for b in range(first_slice, first_slice + n):
        rng = rng_for(cfg_id, b, 5)
        R = float(rng.choice([4.0, 6.0, 8.0]))
        snr = float(rng.uniform(30.0, 45.0))
        out.append(make_slice(cfg_id, b, 256, 256, 16, R, 6.0, 16, snr))
    return out, 4, 50


def workload_c5(n: int, cfg_id: int = 5, first_slice: int = 0):
    """512x512 textured slices for the learned denoiser at scale (evaluation cfg_id 5,
    training 50): workload_batch512's recipe, R alternating 8 and 12."""
    return workload_batch512(n, cfg_id=cfg_id, first_slice=first_slice)


# ---------------------------------------------------------------------------------
# 3D volumes (Section 1: Phi may use a 3D DFT).  Random-ellipsoid phantoms with a
# smooth phase, the polynomial variable density in the normalised 3D radius with a
# fully sampled C x C x C centre, Bernoulli sampling and white complex noise, seeded as
# for slices.  Arrays are [nz][ny][nx].

@dataclass
class Volume:
    x0: np.ndarray       # complex128 [nz][ny][nx]
    y: np.ndarray        # complex128 [nz][ny][nx] zero-filled measurements, natural order
    mask: np.ndarray     # uint8
    p: np.ndarray        # float64
    sigma2: float
    R: float
    snr_db: float


def phantom3d(cfg_id: int, vol_id: int, nz: int, ny: int, nx: int, n_ellipsoids: int) -> np.ndarray:
    w = 2.0 * (np.arange(nz) + 0.5) / nz - 1.0
    v = 2.0 * (np.arange(ny) + 0.5) / ny - 1.0
    u = 2.0 * (np.arange(nx) + 0.5) / nx - 1.0
    W, V, U = np.meshgrid(w, v, u, indexing="ij")
    rng = rng_for(cfg_id, vol_id, STREAM_PHANTOM)
    mag = np.zeros(U.shape)
    for e in range(n_ellipsoids):
        if e == 0:
            c = rng.uniform(-0.1, 0.1, size=3)
            ax = rng.uniform(0.6, 0.85, size=3)
        else:
            c = rng.uniform(-0.5, 0.5, size=3)
            ax = rng.uniform(0.05, 0.4, size=3)
        ang = rng.uniform(0.0, np.pi)   # rotation about the z axis
        inten = rng.uniform(0.1, 1.0)
        du, dv, dw = U - c[0], V - c[1], W - c[2]
        ur = np.cos(ang) * du + np.sin(ang) * dv
        vr = -np.sin(ang) * du + np.cos(ang) * dv
        mag[(ur / ax[0]) ** 2 + (vr / ax[1]) ** 2 + (dw / ax[2]) ** 2 <= 1.0] = inten
    prng = rng_for(cfg_id, vol_id, STREAM_PHASE)
    q = prng.uniform(-1.0, 1.0, size=4)
    phi = q[0] + q[1] * U + q[2] * V + q[3] * W
    pm = np.abs(phi).max()
    if pm > 0:
        phi = phi * (np.pi / 4.0) / pm
    return mag * np.exp(1j * phi)


@functools.lru_cache(maxsize=16)
def _density3d_centred(nz: int, ny: int, nx: int, R: float, d: float, C: int) -> np.ndarray:
    kz = np.arange(-(nz // 2), nz - nz // 2)[:, None, None].astype(np.float64)
    ky = np.arange(-(ny // 2), ny - ny // 2)[None, :, None].astype(np.float64)
    kx = np.arange(-(nx // 2), nx - nx // 2)[None, None, :].astype(np.float64)
    rad = np.sqrt(kz ** 2 + ky ** 2 + kx ** 2)
    base = (1.0 - rad / rad.max()) ** d
    centre = ((np.abs(kz + 0.5) <= C / 2) & (np.abs(ky + 0.5) <= C / 2) & (np.abs(kx + 0.5) <= C / 2))
    target = nz * ny * nx / float(R)
    if target < centre.sum():
        raise ValueError("undersampling factor incompatible with the fully sampled centre")
    lo, hi = -1.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        p = np.clip(base + mid, 0.0, 1.0)
        p[centre] = 1.0
        if p.sum() < target:
            lo = mid
        else:
            hi = mid
    p = np.clip(base + hi, 0.0, 1.0)
    p[centre] = 1.0
    p.setflags(write=False)
    return p


def density3d(nz: int, ny: int, nx: int, R: float, d: float, C: int) -> np.ndarray:
    """p = clip((1 - r)^d + c, 0, 1) in the normalised 3D radius, fully sampled centre
    cube, sum(p) = N / R; natural FFT order."""
    return np.fft.ifftshift(_density3d_centred(nz, ny, nx, float(R), float(d), int(C)))


def make_volume(cfg_id: int, vol_id: int, nz: int, ny: int, nx: int, n_ellipsoids: int, R: float,
                d: float, C: int, snr_db: float) -> Volume:
    x0 = phantom3d(cfg_id, vol_id, nz, ny, nx, n_ellipsoids)
    p = density3d(nz, ny, nx, R, d, C)
    mask = (rng_for(cfg_id, vol_id, STREAM_MASK).random(p.shape) < p).astype(np.uint8)
    N = x0.size
    sigma2 = float(np.sum(np.abs(x0) ** 2) / (N * 10.0 ** (snr_db / 10.0)))
    nrng = rng_for(cfg_id, vol_id, STREAM_NOISE)
    eps = (nrng.standard_normal(p.shape) + 1j * nrng.standard_normal(p.shape)) * np.sqrt(sigma2 / 2.0)
    y = mask * (np.fft.fftn(x0, norm="ortho") + eps)
    return Volume(x0=x0, y=y, mask=mask, p=p, sigma2=sigma2, R=float(R), snr_db=float(snr_db))


def workload_volume32(vol_id: int = 0):
    """32^3 volume, 6 ellipsoids, p ~ (1-r)^4 + c, 4^3 centre, R = 4, 35 dB, 2 Haar levels,
    20 iterations."""
    return [make_volume(60, vol_id, 32, 32, 32, 6, 4.0, 4.0, 4, 35.0)], 2, 20


def workload_volume64(n: int = 1, R: float = 6.0):
    """64^3 volumes, 12 ellipsoids, p ~ (1-r)^6 + c, 8^3 centre, R = 6, 40 dB, 3 Haar
    levels, 30 iterations (finest band 32^3 = 32768 coefficients)."""
    return [make_volume(61, v, 64, 64, 64, 12, R, 6.0, 8, 40.0) for v in range(n)], 3, 30

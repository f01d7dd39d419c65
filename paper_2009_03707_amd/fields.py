"""Seeded synthetic scalar fields on 3D grids.

This module only draws random numbers and evaluates the analytic test fields
(sines, Gaussian random fields, Gaussian blobs).  It holds none of the
Morse-Smale arithmetic and is shared by the test oracle and the GPU path so
that both see bit-identical inputs.

Layout convention used everywhere in this project: a field of vertex counts
(nx, ny, nz) is a C-ordered float32 array of shape (nz, ny, nx); vertex
(x, y, z) has id ``x + nx * (y + ny * z)``.

The paper evaluates on public volume datasets (Open SciVis, Section 5); those
are not available here, so the generators below stand in for them with the
shapes and value structure of the benchmark configurations: a smooth
analytic field, a k^-3 Gaussian random field, a noisy sum of anisotropic
blobs (high critical-point density), batches of uneven non-cubic fields, and
an advected time series with interleaved requests.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

TWO_PI = 2.0 * np.pi


def sha256(a: np.ndarray) -> str:
    """Hex digest of the raw bytes of a C-contiguous array."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def sine_field(n: int = 32, seed: int = 0, noise: float = 1e-3) -> np.ndarray:
    """f = sin(3x) + sin(5y) + sin(7z) on [0, 2pi]^3 (endpoints included),
    n samples per axis, plus uniform noise in [-noise, noise] drawn from
    ``default_rng(seed)``.  Evaluated in float64, returned as float32."""
    t = np.linspace(0.0, TWO_PI, n)
    f = (np.sin(3.0 * t)[None, None, :] + np.sin(5.0 * t)[None, :, None]
         + np.sin(7.0 * t)[:, None, None])
    if noise > 0:
        rng = np.random.default_rng(seed)
        f = f + rng.uniform(-noise, noise, size=f.shape)
    return np.ascontiguousarray(f.astype(np.float32))


def grf_field(dims, seed: int = 0, power: float = 3.0) -> np.ndarray:
    """Gaussian random field with power spectrum |k|^-power on a periodic box
    of vertex counts dims = (nx, ny, nz): white noise from
    ``default_rng(seed).standard_normal``, filtered by |k|^(-power/2) in
    Fourier space (k = 0 removed), then normalised to zero mean and unit
    variance.  Float64 internally, float32 out."""
    nx, ny, nz = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx))
    fw = np.fft.rfftn(w)
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    with np.errstate(divide="ignore"):
        amp = np.where(k > 0, k ** (-power / 2.0), 0.0)
    f = np.fft.irfftn(fw * amp, s=(nz, ny, nx), axes=(0, 1, 2))
    f = (f - f.mean()) / f.std()
    return np.ascontiguousarray(f.astype(np.float32))


def blob_field(dims, nblobs: int = 2000, seed: int = 0, noise_sigma: float = 0.01,
               sigma_range=(2.0, 20.0)) -> np.ndarray:
    """Sum of ``nblobs`` axis-aligned anisotropic Gaussian blobs plus
    N(0, noise_sigma) noise.

    Draw order from ``default_rng(seed)``: centres U[0, n) per axis
    (shape (nblobs, 3), columns x, y, z), amplitudes U[-1, 1] (nblobs),
    sigmas U[sigma_range] per axis (nblobs, 3), then the noise volume.
    Each blob is evaluated separably over a +-4 sigma window clipped to the
    grid.  Float64 internally, float32 out."""
    nx, ny, nz = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(nblobs, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    amps = rng.uniform(-1.0, 1.0, size=nblobs)
    sig = rng.uniform(sigma_range[0], sigma_range[1], size=(nblobs, 3))
    f = np.zeros((nz, ny, nx), dtype=np.float64)
    for b in range(nblobs):
        cx, cy, cz = centres[b]
        sx, sy, sz = sig[b]
        lo = [max(0, int(np.floor(c - 4.0 * s))) for c, s in ((cx, sx), (cy, sy), (cz, sz))]
        hi = [min(n, int(np.ceil(c + 4.0 * s)) + 1) for c, s, n in ((cx, sx, nx), (cy, sy, ny), (cz, sz, nz))]
        if hi[0] <= lo[0] or hi[1] <= lo[1] or hi[2] <= lo[2]:
            continue
        gx = np.exp(-0.5 * ((np.arange(lo[0], hi[0]) - cx) / sx) ** 2)
        gy = np.exp(-0.5 * ((np.arange(lo[1], hi[1]) - cy) / sy) ** 2)
        gz = np.exp(-0.5 * ((np.arange(lo[2], hi[2]) - cz) / sz) ** 2)
        f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += amps[b] * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    if noise_sigma > 0:
        f += rng.normal(0.0, noise_sigma, size=f.shape)
    return np.ascontiguousarray(f.astype(np.float32))


def random_field(dims, seed: int = 0, levels: int = 0) -> np.ndarray:
    """I.i.d. U[0,1) values; with ``levels`` > 0 they are quantised to that
    many distinct values, which produces many exact ties (exercising the
    vertex-id tie break)."""
    nx, ny, nz = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.0, 1.0, size=(nz, ny, nx))
    if levels > 0:
        f = np.floor(f * levels)
    return np.ascontiguousarray(f.astype(np.float32))


@dataclass
class BatchItem:
    dims: tuple
    kind: str
    seed: int


def batch_specs(count: int = 64, seed0: int = 1000, lo: int = 64, hi: int = 320):
    """Specs of the uneven batch: field i uses ``default_rng(seed0 + i)``;
    its sides are drawn U{lo..hi} independently per axis (x, y, z) from that
    generator, even i are k^-3 GRFs, odd i are blob fields whose blob count
    is 2000 scaled by volume relative to 512^3 (at least 1)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        dims = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        out.append(BatchItem(dims=dims, kind="grf" if i % 2 == 0 else "blobs", seed=seed0 + i))
    return out


def make_batch_field(item: BatchItem) -> np.ndarray:
    nx, ny, nz = item.dims
    if item.kind == "grf":
        return grf_field(item.dims, seed=item.seed)
    nb = max(1, int(round(2000.0 * nx * ny * nz / float(512 ** 3))))
    return blob_field(item.dims, nblobs=nb, seed=item.seed)


def make_batch(specs, workers: int = 0):
    """All fields of a batch, generated in a process pool (order kept)."""
    import concurrent.futures as cf
    import os
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1:
        return [make_batch_field(s) for s in specs]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(make_batch_field, specs))


def advected_step(base: np.ndarray, t: int) -> np.ndarray:
    """Timestep t of the advected series: the periodic base field shifted by
    t voxels along x (constant velocity of one voxel per step)."""
    return np.ascontiguousarray(np.roll(base, t, axis=2))


def request_arrivals(duration_s: float, rate: float = 20.0, seed: int = 7,
                     lo: int = 64, hi: int = 256):
    """Poisson request stream: exponential gaps of mean 1/rate drawn from
    ``default_rng(seed)``, each request cubic with side U{lo..hi}; kinds
    alternate GRF / blobs.  Returns a list of (arrival_s, side, kind, seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            break
        side = int(rng.integers(lo, hi + 1))
        out.append((t, side, "grf" if i % 2 == 0 else "blobs", 10_000 + i))
        i += 1
    return out

"""Seeded synthetic fields shaped like the paper's workloads.

The paper evaluates on SDRBench-type simulation outputs (JHTDB and Nyx 512^3,
Miranda 256x384x384, RTM, QMCPack, S3D 500^3; Table II).  Those files are not
available here, so these generators stand in for them: smooth fields with
power-law spectra, climate-like 2D fields with fill values, and sharp fronts.
Nothing here computes any part of the compression method; the module only
draws random numbers (numpy PCG64, float64) and returns float32 arrays.
"""
from __future__ import annotations

import math

import numpy as np

try:  # multithreaded FFT when available; results do not depend on threads
    import scipy.fft as _fft

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=-1)
except Exception:  # pragma: no cover
    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def bumps_field(shape=(64, 64, 64), seed=1, noise=1e-4) -> np.ndarray:
    """Sum of 8 Gaussian bumps, 3 low-frequency sinusoids and N(0, noise)."""
    rng = np.random.default_rng(seed)
    D = len(shape)
    axes = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    f = np.zeros(shape, dtype=np.float64)
    for _ in range(8):
        amp = rng.uniform(-1.0, 1.0)
        ctr = rng.uniform(0.0, 1.0, size=D) * np.array(shape)
        sig = rng.uniform(3.0, 12.0)
        r2 = sum((axes[d] - ctr[d]) ** 2 for d in range(D))
        f += amp * np.exp(-r2 / (2.0 * sig * sig))
    ks = [k for k in np.ndindex(*([3] * D)) if any(k)]
    for _ in range(3):
        k = ks[rng.integers(len(ks))]
        B = rng.uniform(0.2, 0.5)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        arg = sum(2.0 * math.pi * k[d] * axes[d] / shape[d] for d in range(D))
        f += B * np.sin(arg + phi)
    f += rng.normal(0.0, noise, size=shape)
    return f.astype(np.float32)


def spectral_field(shape, beta=5.0 / 3.0, seed=2, mean=0.0, std=1.0) -> np.ndarray:
    """Random-phase Gaussian field with |F(k)| = |k|^-(beta+D-1)/2.

    The power per shell then falls as k^-beta (e.g. beta = 5/3, the
    Kolmogorov slope of turbulence data such as JHTDB)."""
    rng = np.random.default_rng(seed)
    D = len(shape)
    freqs = [np.fft.fftfreq(s) * s for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    k2 = np.zeros([len(f) for f in freqs], dtype=np.float32)
    for d, f in enumerate(freqs):
        sh = [1] * D
        sh[d] = len(f)
        k2 += (f.astype(np.float32) ** 2).reshape(sh)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 >= 1.0, k2 ** np.float32(-(beta + D - 1) / 4.0), np.float32(0.0))
    del k2
    phase = rng.uniform(0.0, 2.0 * math.pi, size=amp.shape).astype(np.float32)
    spec = (amp * np.exp(1j * phase)).astype(np.complex64)
    del amp, phase
    f = _irfftn(spec, shape)
    del spec
    f = f.astype(np.float64)
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f /= sd
    return (f * std + mean).astype(np.float32)


def climate_field(seed, shape=(1800, 3600), fill=-999.0, fill_frac=0.05) -> np.ndarray:
    """2D lat-lon field: zonal cosines in latitude plus a k^-3 perturbation
    (std 2); a blob-shaped 5 % of cells carries a constant fill value."""
    rng = np.random.default_rng(seed)
    ny, nx = shape
    lat = (np.arange(ny, dtype=np.float64) + 0.5) / ny * math.pi - math.pi / 2.0
    zonal = np.zeros(ny)
    for m in range(1, 4):
        a = rng.uniform(2.0, 10.0)
        psi = rng.uniform(0.0, 2.0 * math.pi)
        zonal += a * np.cos(2 * m * lat + psi)
    s1, s2 = rng.integers(1 << 30, size=2)
    pert = spectral_field(shape, beta=3.0, seed=int(s1), std=2.0).astype(np.float64)
    f = zonal[:, None] + pert
    mask_src = spectral_field(shape, beta=3.0, seed=int(s2))
    thr = np.quantile(mask_src, fill_frac)
    f[mask_src <= thr] = fill
    return f.astype(np.float32)


def front_field(shape, seed, width=2.0) -> np.ndarray:
    """Sharp front 5 tanh(n.(r - r0) / width) on an oblique seeded normal,
    plus a k^-3 perturbation of std 0.05."""
    rng = np.random.default_rng(seed)
    D = len(shape)
    nrm = rng.normal(size=D)
    nrm /= np.linalg.norm(nrm)
    r0 = rng.uniform(0.3, 0.7, size=D) * np.array(shape)
    s = np.zeros(shape, dtype=np.float64)
    for d in range(D):
        sh = [1] * D
        sh[d] = shape[d]
        s = s + (nrm[d] * (np.arange(shape[d]) - r0[d])).reshape(sh)
    f = 5.0 * np.tanh(s / width)
    f += spectral_field(shape, beta=3.0, seed=int(rng.integers(1 << 30)), std=0.05)
    return f.astype(np.float32)


# ---------------------------------------------------------------- workloads
def fib_spikes(shape, n=24, seed=26) -> np.ndarray:
    """Zeros with spikes of height k at F(k) points (F the Fibonacci numbers
    1, 1, 2, 3, ..., k = 1..n), placed at seeded random points whose
    coordinates are all odd."""
    x = np.zeros(shape, np.float32)
    idx = np.stack(np.meshgrid(*[np.arange(1, s, 2) for s in shape], indexing="ij"),
                   -1).reshape(-1, len(shape))
    np.random.default_rng(seed).shuffle(idx)
    f = [1, 1]
    while len(f) < n:
        f.append(f[-1] + f[-2])
    if sum(f) > len(idx):
        raise ValueError("shape %s has too few all-odd points for %d spike heights" % (shape, n))
    k0 = 0
    for k, c in enumerate(f, 1):
        x[tuple(idx[k0:k0 + c].T)] = np.float32(k)
        k0 += c
    return x


def workload_small(seed=1):
    """64^3 smooth field: bumps + sinusoids + N(0, 1e-4)."""
    return bumps_field((64, 64, 64), seed=seed)


def workload_large(seed=2, shape=(512, 512, 512)):
    """512^3 turbulence-like field (k^-5/3) with a mean offset of 10."""
    return spectral_field(shape, beta=5.0 / 3.0, seed=seed, mean=10.0)


def climate_batch(count=24, shape=(1800, 3600), seed0=300):
    """24 climate-like 2D fields with 5 % fill."""
    return [climate_field(seed0 + i, shape) for i in range(count)]


def uneven_batch(seed0=400, n_a=13, shape_a=(100, 500, 500), n_b=6, shape_b=(256, 384, 384)):
    """13 x 100x500x500 and 6 x 256x384x384 fields: slopes alternate 5/3
    (even index) and 3 (odd); the first field of the second group is a sharp
    front.  Returns (fields, rel_ebs) with eb cycling 1e-2, 1e-3, 1e-4."""
    fields, ebs = [], []
    ebc = [1e-2, 1e-3, 1e-4]
    for i in range(n_a + n_b):
        shape = shape_a if i < n_a else shape_b
        seed = seed0 + i
        if i == n_a:
            f = front_field(shape, seed)
        else:
            f = spectral_field(shape, beta=5.0 / 3.0 if i % 2 == 0 else 3.0, seed=seed)
        fields.append(f)
        ebs.append(ebc[i % 3])
    return fields, ebs

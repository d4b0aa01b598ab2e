"""Random permeability fields (stand-ins for the paper's SGeMS sets).

The paper draws log-normal permeability realisations by sequential Gaussian
simulation (Sec. 4, Table "permeability sets").  Those realisations are not
available, so stationary Gaussian fields are drawn here instead by circulant
embedding: the covariance is sampled on a periodic grid padded well beyond the
correlation length, its FFT gives the spectral density, and white noise is
coloured with its square root.  Arrays are returned in (nz, ny, nx) order so
that C-order flattening gives the cell index i + nx*(j + ny*k).
"""

from __future__ import annotations

import numpy as np


def _as_triple(v, ndim):
    if np.isscalar(v):
        return (float(v),) * ndim
    v = tuple(float(x) for x in v)
    assert len(v) == ndim
    return v


def gaussian_field(shape, corr_len, seed):
    """Zero-mean, unit-variance stationary Gaussian field.

    shape: (nz, ny, nx) or (ny, nx).  corr_len: per-axis correlation length in
    cells (same order as shape, or a scalar).  Covariance exp(-|h/l|_2).
    """
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    ell = _as_triple(corr_len, ndim)
    rng = np.random.default_rng(seed)
    padded = tuple(int(n + 4 * max(l, 1.0)) for n, l in zip(shape, ell))
    # periodic lag per axis
    lag2 = np.zeros(padded)
    for ax, (m, l) in enumerate(zip(padded, ell)):
        h = np.arange(m, dtype=np.float64)
        h = np.minimum(h, m - h) / max(l, 1e-12)
        sh = [1] * ndim
        sh[ax] = m
        lag2 = lag2 + (h.reshape(sh) ** 2)
    cov = np.exp(-np.sqrt(lag2))
    spec = np.fft.fftn(cov).real
    spec = np.clip(spec, 0.0, None)
    noise = rng.standard_normal(padded)
    field = np.fft.ifftn(np.sqrt(spec) * np.fft.fftn(noise)).real
    field = field[tuple(slice(0, n) for n in shape)]
    field = field - field.mean()
    sd = field.std()
    if sd > 0:
        field = field / sd
    return np.ascontiguousarray(field)


def lognormal_permeability(shape, mean_lnk, sigma_lnk, corr_len, seed):
    """k = exp(mean + sigma * z) with z from gaussian_field."""
    z = gaussian_field(shape, corr_len, seed)
    return np.exp(mean_lnk + sigma_lnk * z)


def channel_permeability(shape, seed, k_channel=1.0, k_matrix=1e-4,
                         fraction=0.30, width=(4, 12), height=(4, 12),
                         amplitude=(4.0, 32.0), wavelength=(64.0, 256.0)):
    """Binary channelised field: sinusoidal channels along x.

    Channels of k_channel are added to a k_matrix background until the channel
    volume fraction reaches `fraction`.  Each channel has centreline
    y_c(x) = y0 + A sin(2 pi x / lam + phase), a width drawn from `width`
    cells and a vertical extent drawn from `height` cells.
    shape: (nz, ny, nx).
    """
    nz, ny, nx = (int(s) for s in shape)
    rng = np.random.default_rng(seed)
    inside = np.zeros((nz, ny, nx), dtype=bool)
    x = np.arange(nx, dtype=np.float64)
    yy = np.arange(ny, dtype=np.float64)[:, None]
    total = nz * ny * nx
    guard = 0
    while inside.sum() < fraction * total and guard < 10000:
        guard += 1
        w = int(rng.integers(width[0], width[1] + 1))
        h = int(rng.integers(height[0], height[1] + 1))
        amp = rng.uniform(*amplitude)
        lam = rng.uniform(*wavelength)
        phase = rng.uniform(0, 2 * np.pi)
        y0 = rng.uniform(0, ny)
        z0 = int(rng.integers(0, max(1, nz - h + 1)))
        yc = y0 + amp * np.sin(2 * np.pi * x / lam + phase)  # (nx,)
        band = np.abs(yy - yc[None, :]) <= (w / 2.0)            # (ny, nx)
        trial = inside.copy()
        trial[z0:z0 + h] |= band[None, :, :]
        if trial.sum() > (fraction + 0.01) * total:
            # trim the last channel's vertical extent to stay within tolerance
            for hh in range(h - 1, 0, -1):
                trial = inside.copy()
                trial[z0:z0 + hh] |= band[None, :, :]
                if trial.sum() <= (fraction + 0.01) * total:
                    break
        inside = trial
    return np.where(inside, k_channel, k_matrix).astype(np.float64)

"""Seeded permeability and porosity fields on an nx x ny x nz Cartesian grid.

Arrays are returned flattened in the natural cell order c = i + nx*(j + ny*k)
(x fastest), the order used by every matrix in this project.

Recipes (synthetic stand-ins for the paper's homogeneous and SPE10 fields):
  * iid:         ln k ~ N(ln k_mean, sigma^2) independently per cell;
  * gaussian:    ln k = ln k_mean + sigma*g, g a white-noise field filtered in
                 Fourier space to the covariance exp(-(r/l)^2) (l in cells,
                 possibly anisotropic), then standardised to mean 0, std 1;
  * channelised: binary facies, channel where g exceeds its (1-frac)
                 quantile; k = k_channel there, k_background elsewhere.
Porosity is iid U(0.15, 0.25) in every case.
"""
import numpy as np

MILLIDARCY = 9.869233e-16  # m^2


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_field(shape_xyz, corr_len, rng):
    """Standardised Gaussian random field with covariance exp(-(r/l)^2).

    shape_xyz = (nx, ny, nz); corr_len is a scalar or an (lx, ly, lz) tuple in
    cells.  Periodic FFT filtering of white noise by the square root of the
    spectral density exp(-|k l|^2 / 4)."""
    nx, ny, nz = shape_xyz
    if np.isscalar(corr_len):
        corr_len = (corr_len, corr_len, corr_len)
    noise = rng.standard_normal((nz, ny, nx))
    f = np.fft.rfftn(noise)
    kz = 2 * np.pi * np.fft.fftfreq(nz)[:, None, None]
    ky = 2 * np.pi * np.fft.fftfreq(ny)[None, :, None]
    kx = 2 * np.pi * np.fft.rfftfreq(nx)[None, None, :]
    lx, ly, lz = corr_len
    amp = np.exp(-((kx * lx) ** 2 + (ky * ly) ** 2 + (kz * lz) ** 2) / 8.0)
    g = np.fft.irfftn(f * amp, s=(nz, ny, nx), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    return g.reshape(-1)


def make_fields(shape_xyz, kind, seed, sigma=1.0, corr_len=8.0,
                k_mean_md=100.0, channel_frac=0.2, k_channel_md=1.0e4,
                k_background_md=1.0):
    """Return (perm [m^2], porosity) flattened in natural order."""
    nx, ny, nz = shape_xyz
    n = nx * ny * nz
    rng = _rng(seed)
    if kind == "iid":
        lnk = np.log(k_mean_md) + sigma * rng.standard_normal(n)
        perm = np.exp(lnk) * MILLIDARCY
    elif kind == "gaussian":
        g = gaussian_field(shape_xyz, corr_len, rng)
        perm = np.exp(np.log(k_mean_md) + sigma * g) * MILLIDARCY
    elif kind == "channelised":
        g = gaussian_field(shape_xyz, corr_len, rng)
        thr = np.quantile(g, 1.0 - channel_frac)
        perm = np.where(g > thr, k_channel_md, k_background_md) * MILLIDARCY
    elif kind == "constant":
        perm = np.full(n, k_mean_md * MILLIDARCY)
    else:
        raise ValueError(f"unknown field kind {kind!r}")
    poro = rng.uniform(0.15, 0.25, n)
    return perm, poro

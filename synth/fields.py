"""Input recipes (see the design notes for the configurations they serve).

* ``filtered_eigenstrain``: i.i.d. N(0, 1) per component and layer, filtered
  in-plane by an isotropic amplitude |k|^-2 (integer wavenumbers, k = 0 -> 0),
  multiplied by exp(-z / decay) in depth and scaled to a given max |value|.
* ``filtered_traction``: the same in-plane filter on 3 components.
* ``paraboloid``: rigid paraboloid h = -|x - x_c|^2 / (2R) with the
  minimum-image distance in the periodic cell (contact at the centre node).
* ``rough_surface``: self-affine periodic surface by spectral filtering,
  amplitude sqrt(C(|k|)) with C = 1 on the plateau k_r <= |k| < k_l... see
  the docstring; random phases; rms spectral slope normalisation; returned
  as h - max h so that the highest asperity touches first.
* ``poisson_requests``: seeded arrival times and per-request parameters for
  the continuous-batching server.
"""
import numpy as np


def grid_dict(nx, ny, nz, lx=1.0, ly=1.0, lz=0.25):
    return {"nx": int(nx), "ny": int(ny), "nz": int(nz),
            "lx": float(lx), "ly": float(ly), "lz": float(lz)}


def _kmag(nx, ny):
    kx = np.fft.fftfreq(nx, d=1.0 / nx)
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    return np.hypot(kx[None, :], ky[:, None])


def _filter_planes(noise, power):
    ny, nx = noise.shape[-2:]
    k = _kmag(nx, ny)
    amp = np.zeros_like(k)
    nzk = k > 0
    amp[nzk] = k[nzk] ** (-power)
    spec = np.fft.fft2(noise, axes=(-2, -1)) * amp
    return np.real(np.fft.ifft2(spec, axes=(-2, -1)))


def filtered_eigenstrain(grid, seed=0, decay=0.1, max_abs=1e-3, power=2.0, layers=None):
    """(6, nz, ny, nx) float64 plastic strain field.  layers: optional list
    of depth indices that receive the filtered field (others stay zero), for
    inputs of full-size grids that are cheap to generate."""
    nx, ny, nz, lz = grid["nx"], grid["ny"], grid["nz"], grid["lz"]
    rng = np.random.default_rng(seed)
    z = np.linspace(0.0, lz, nz)
    if layers is None:
        noise = rng.standard_normal((6, nz, ny, nx))
        f = _filter_planes(noise, power)
        f = f * np.exp(-z / decay)[None, :, None, None]
    else:
        layers = list(layers)
        part = _filter_planes(rng.standard_normal((6, len(layers), ny, nx)), power)
        part = part * np.exp(-z[layers] / decay)[None, :, None, None]
        f = np.zeros((6, nz, ny, nx))
        f[:, layers] = part
    m = np.max(np.abs(f))
    return np.ascontiguousarray(f * (max_abs / m if m > 0 else 1.0))


def filtered_traction(grid, seed=1000, max_abs=1e-2, power=2.0):
    """(3, ny, nx) float64 surface traction."""
    nx, ny = grid["nx"], grid["ny"]
    rng = np.random.default_rng(seed)
    f = _filter_planes(rng.standard_normal((3, ny, nx)), power)
    m = np.max(np.abs(f))
    return np.ascontiguousarray(f * (max_abs / m if m > 0 else 1.0))


def paraboloid(grid, R=0.5, center=None):
    """(ny, nx) profile -|x - x_c|^2/(2R), periodic minimum image."""
    nx, ny, lx, ly = grid["nx"], grid["ny"], grid["lx"], grid["ly"]
    if center is None:
        center = (0.5 * lx, 0.5 * ly)
    x = np.arange(nx) * lx / nx
    y = np.arange(ny) * ly / ny
    dx = x - center[0]
    dy = y - center[1]
    dx = dx - lx * np.round(dx / lx)
    dy = dy - ly * np.round(dy / ly)
    r2 = dx[None, :] ** 2 + dy[:, None] ** 2
    return np.ascontiguousarray(-r2 / (2.0 * R))


def rough_surface(nx, ny, hurst=0.8, k_roll=4, k_cut=None, rms_slope=0.1,
                  seed=0, lx=1.0, ly=1.0):
    """(ny, nx) self-affine surface, contact profile h - max(h).

    PSD C(|k|) = 1 for 1 <= |k| < k_roll, (|k|/k_roll)^(-2(1+H)) for
    k_roll <= |k| <= k_cut, 0 otherwise (integer wavenumbers, circular
    cut-offs); amplitude sqrt(C); uniform random phases, made Hermitian by
    taking the real part of the inverse transform of a full random spectrum.
    Normalised so the spectral rms slope sqrt(sum |q|^2 |h_k|^2) equals
    rms_slope, q = 2 pi k / L.
    """
    if k_cut is None:
        k_cut = min(nx, ny) // 4
    rng = np.random.default_rng(seed)
    k = _kmag(nx, ny)
    psd = np.zeros_like(k)
    plateau = (k >= 1) & (k < k_roll)
    tail = (k >= k_roll) & (k <= k_cut)
    psd[plateau] = 1.0
    psd[tail] = (k[tail] / k_roll) ** (-2.0 * (1.0 + hurst))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx))
    spec = np.sqrt(psd) * np.exp(1j * phase)
    h = np.real(np.fft.ifft2(spec)) * (nx * ny)
    hk = np.fft.fft2(h) / (nx * ny)
    kx = np.fft.fftfreq(nx, d=1.0 / nx) * 2 * np.pi / lx
    ky = np.fft.fftfreq(ny, d=1.0 / ny) * 2 * np.pi / ly
    q2 = kx[None, :] ** 2 + ky[:, None] ** 2
    slope = np.sqrt(np.sum(q2 * np.abs(hk) ** 2))
    h = h * (rms_slope / slope)
    return np.ascontiguousarray(h - h.max())


GRIDS_SERVING = ((64, 64, 32), (128, 128, 64), (256, 256, 64), (512, 512, 96))


def poisson_requests(n=256, rate=100.0, seed=2024, grids=GRIDS_SERVING):
    """List of dicts: arrival time, grid, Hurst exponent, mean pressure, seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        g = grids[rng.integers(len(grids))]
        out.append({"id": i, "arrival": float(t[i]), "nx": g[0], "ny": g[1], "nz": g[2],
                    "hurst": float(rng.uniform(0.5, 0.9)),
                    "pbar": float(rng.uniform(0.005, 0.05)),
                    "seed": int(rng.integers(1 << 31))})
    return out

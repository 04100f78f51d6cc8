"""Frictionless normal contact with a rigid surface under total load (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. 5.1: with the plastic strain frozen, the contact problem is the Kalker
dual minimisation of the surface energy over admissible pressures:
minimise  Phi(p) = 1/2 p.M p - h.p  subject to  p >= 0,  dA sum p = W
(eqn total_pressure), where M is the periodic surface compliance of the
half-space, u3 = M[p] at z = 0.  Per in-plane mode M is 2 / (E* |q|)
(k = 0 dropped: the mean displacement is free and fixed by the load), which
is the z = 0 normal displacement of the Boussinesq-Cerruti solution for a
normal surface load.  The gradient of Phi is g = u3 - h; at the minimiser
g equals a constant (minus the rigid approach) on the contact set and is not
below it elsewhere.

The paper solves this with the projected conjugate gradient of Polonsky and
Keer (1999) (it only names the method); the steps below follow that
published algorithm, load-controlled: CG on the current contact set with the
mean gap over the set removed, projection onto p >= 0, re-admission of
points whose gap says they should carry load (with a restart of the
conjugation), and renormalisation to the prescribed load.
"""
import numpy as np

from . import elastic


def surface_compliance_symbol(grid, E, nu):
    """2 / (E* |q|) on the full (ny, nx) DFT grid, 0 at k = 0."""
    nx, ny = grid['nx'], grid['ny']
    k1 = np.fft.fftfreq(nx, d=1.0 / nx) * 2 * np.pi / grid['lx']
    k2 = np.fft.fftfreq(ny, d=1.0 / ny) * 2 * np.pi / grid['ly']
    q = np.hypot(k1[None, :], k2[:, None])
    sym = np.zeros_like(q)
    sym[q > 0] = 2.0 / (elastic.e_star(E, nu) * q[q > 0])
    return sym


def apply_compliance(p, sym):
    return np.real(np.fft.ifft2(np.fft.fft2(p) * sym))


def contact_solve(h, W, grid, E, nu, tol=1e-14, max_iter=5000, p0=None):
    """Polonsky-Keer projected CG.  h: (ny, nx) rigid surface along +e3.

    Returns (p, gap, info): p >= 0 with dA sum p = W; gap = u3 - h minus its
    mean over the contact set (>= 0, 0 on the contact set at convergence)."""
    h = np.asarray(h, dtype=float)
    nx, ny = grid['nx'], grid['ny']
    n = nx * ny
    dA = grid['lx'] * grid['ly'] / n
    sym = surface_compliance_symbol(grid, E, nu)
    # diagonal of the compliance matrix: the surface displacement under a
    # unit point force at its own point, the mean of the symbol over modes
    m_diag = float(np.mean(sym))
    if p0 is None or not np.any(p0):
        p = np.full((ny, nx), W / (n * dA))
    else:
        p = np.array(p0, dtype=float)
        p *= W / (dA * p.sum())
    t = np.zeros_like(p)
    G_old = 1.0
    delta = 0.0
    err = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        Ic = p > 0
        g = apply_compliance(p, sym) - h
        g = g - g[Ic].mean()
        G = np.sum(g[Ic] ** 2)
        beta = delta * G / G_old if G_old > 0 else 0.0
        t = np.where(Ic, g + beta * t, 0.0)
        G_old = G
        r = apply_compliance(t, sym)
        r = r - r[Ic].mean()
        den = np.sum(r[Ic] * t[Ic])
        tau = np.sum(g[Ic] * t[Ic]) / den if den != 0 else 0.0
        p_old = p
        p = p - tau * t
        p = np.maximum(p, 0.0)
        Iol = (p == 0) & (g < 0)
        if np.any(Iol):
            delta = 0.0
            # points that overlap the surface re-enter with a pressure
            # proportional to their overlap; when the conjugate-gradient
            # step vanishes (the gap is already uniform on the contact set,
            # e.g. a set of one point) the published update would re-admit
            # nothing, and the step of a point load, 1 / M_ii, is taken
            step = tau if tau != 0.0 else 1.0 / m_diag
            p[Iol] = p[Iol] - step * g[Iol]
        else:
            delta = 1.0
        p = p * (W / (dA * p.sum()))
        err = dA * np.sum(np.abs(p - p_old)) / W
        if err < tol:
            break
    Ic = p > 0
    g = apply_compliance(p, sym) - h
    gap = g - g[Ic].mean()
    info = {"iters": it, "rel_change": err, "contact_fraction": float(np.mean(Ic)),
            "kkt_residual": kkt_residual(p, gap, h)}
    return p, gap, info


def kkt_residual(p, gap, h):
    """max(|gap| on the contact set, -min gap) relative to the profile scale."""
    Ic = p > 0
    scale = max(np.max(np.abs(h)), 1e-300)
    on = np.max(np.abs(gap[Ic])) if np.any(Ic) else 0.0
    off = max(0.0, -np.min(gap))
    return float(max(on, off) / scale)

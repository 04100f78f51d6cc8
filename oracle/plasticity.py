"""J2 plasticity and the incremental volume-integral fixed point (oracle).

Test infrastructure only (see ``oracle/__init__``).

* ``return_map``: von Mises yield f_y(sigma) = sqrt(3/2)|s| (Sec. 4.1) with
  linear isotropic hardening f_h(e_p) = sigma_y + E_h e_p, associated flow
  d eps_p = (3 d e_p / (2 f_y)) s.  The paper gives the model, not the
  integration algorithm; this is the backward-Euler radial return, exact for
  linear hardening: trial stress, then if f = f_y(sigma_tr) - f_h(e_p_n) > 0
  the consistency condition f_y(sigma_tr) - 3 mu d_ep = f_h(e_p_n + d_ep)
  gives d_ep = f / (3 mu + E_h) along the trial deviator.
* ``return_map_tangent``: the directional derivative of d_eps_p(d_eps) in a
  direction v (the consistent tangent the paper notes is known for the
  implicit scheme of Sec. 4.2, used by the Newton-Krylov alternative it
  mentions in Sec. 4.3): the chain rule through the radial return above,
  zero where the trial state is elastic.
* ``residual``: R[d_eps] = d_eps - grad_s M[dT] - grad_s N[C : d_eps_p(d_eps; S_n)]
  (eqn incremental_strain and the residual that follows it).
* ``dfsane``: the spectral-residual iteration of Sec. 4.3
  (d = -alpha sigma R, sigma = |s|^2 / <y, s>) with the nonmonotone line
  search of La Cruz, Martinez and Raydan (2006), which the paper defers to.

Norms and inner products are trapezoid-in-depth weighted Frobenius sums over
the grid (off-diagonal stored components count twice).
"""
import numpy as np

from . import elastic
from . import operators


def return_map(d_eps, sigma_n, ep_n, E, nu, sigma_y0, E_h):
    """Pointwise radial return.  d_eps, sigma_n: (6, ...); ep_n: (...).

    Returns (d_eps_p, d_ep, sigma_np1) with the same shapes."""
    lam, mu = elastic.lame(E, nu)
    d_eps = np.asarray(d_eps, dtype=float)
    sig_tr = np.asarray(sigma_n, dtype=float) + elastic.hooke(d_eps, E, nu)
    mean = (sig_tr[0] + sig_tr[1] + sig_tr[2]) / 3.0
    s = sig_tr.copy()
    s[0] -= mean
    s[1] -= mean
    s[2] -= mean
    w = elastic.VOIGT_WEIGHT.reshape((6,) + (1,) * (s.ndim - 1))
    seq = np.sqrt(1.5 * np.sum(w * s * s, axis=0))
    f = seq - (sigma_y0 + E_h * np.asarray(ep_n, dtype=float))
    flow = f > 0.0
    d_ep = np.where(flow, f / (3.0 * mu + E_h), 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        fac = np.where(flow, 1.5 * d_ep / seq, 0.0)
    d_eps_p = fac * s
    sigma_np1 = sig_tr - 2.0 * mu * d_eps_p
    return d_eps_p, d_ep, sigma_np1


def return_map_tangent(d_eps, sigma_n, ep_n, E, nu, sigma_y0, E_h, v):
    """d/dt d_eps_p(d_eps + t v) at t = 0, stored components on axis 0.

    With s = dev(sigma_n + C : d_eps), f_y = sqrt(3/2)|s|,
    d_ep = (f_y - f_h) / (3 mu + E_h) and d_eps_p = (3 d_ep / (2 f_y)) s,
    a change v of the strain increment changes s by ds = 2 mu dev(v), f_y by
    (3/2) <s, ds> / f_y, d_ep by that over (3 mu + E_h), and d_eps_p by the
    product rule.  Where f <= 0 the return is the identity and the
    derivative is zero (on f = 0 exactly, the one-sided elastic branch)."""
    lam, mu = elastic.lame(E, nu)
    d_eps = np.asarray(d_eps, dtype=float)
    v = np.asarray(v, dtype=float)
    sig_tr = np.asarray(sigma_n, dtype=float) + elastic.hooke(d_eps, E, nu)
    s = _dev(sig_tr)
    ds = _dev(elastic.hooke(v, E, nu))
    w = elastic.VOIGT_WEIGHT.reshape((6,) + (1,) * (s.ndim - 1))
    seq = np.sqrt(1.5 * np.sum(w * s * s, axis=0))
    f = seq - (sigma_y0 + E_h * np.asarray(ep_n, dtype=float))
    flow = f > 0.0
    with np.errstate(invalid="ignore", divide="ignore"):
        dseq = np.where(flow, 1.5 * np.sum(w * s * ds, axis=0) / seq, 0.0)
        d_ep = np.where(flow, f / (3.0 * mu + E_h), 0.0)
        dd_ep = dseq / (3.0 * mu + E_h)
        fac = np.where(flow, 1.5 * d_ep / seq, 0.0)
        dfac = np.where(flow, 1.5 * (dd_ep * seq - d_ep * dseq) / (seq * seq), 0.0)
    return dfac * s + fac * ds


def _dev(t):
    mean = (t[0] + t[1] + t[2]) / 3.0
    out = np.array(t, dtype=float)
    out[0] -= mean
    out[1] -= mean
    out[2] -= mean
    return out


def von_mises(sigma):
    """f_y(sigma) = sqrt(3/2) |dev sigma| for stored components on axis 0."""
    mean = (sigma[0] + sigma[1] + sigma[2]) / 3.0
    s = np.array(sigma, dtype=float)
    s[0] -= mean
    s[1] -= mean
    s[2] -= mean
    w = elastic.VOIGT_WEIGHT.reshape((6,) + (1,) * (s.ndim - 1))
    return np.sqrt(1.5 * np.sum(w * s * s, axis=0))


def depth_weights(nz, lz, z=None):
    """Trapezoid weights of the depth nodes (uniform, or the nodes z)."""
    if z is not None:
        h = np.diff(np.asarray(z, dtype=float))
        w = np.zeros(nz)
        w[:-1] += 0.5 * h
        w[1:] += 0.5 * h
        return w
    h = lz / (nz - 1)
    w = np.full(nz, h)
    w[0] = w[-1] = 0.5 * h
    return w


def inner(a, b, grid):
    """<a, b>: Frobenius over stored components, trapezoid in depth,
    cell area per in-plane point."""
    nz = grid['nz']
    wz = depth_weights(nz, grid['lz'], grid.get('z'))
    da = grid['lx'] * grid['ly'] / (grid['nx'] * grid['ny'])
    wc = elastic.VOIGT_WEIGHT[:, None, None, None]
    return float(np.sum(wc * wz[None, :, None, None] * a * b) * da)

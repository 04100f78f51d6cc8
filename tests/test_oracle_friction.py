"""Pins of the oracle's tangential (frictional) contact solve (CPU only):
the compliance against the pinned Boussinesq-Cerruti operator, the
Cattaneo-Mindlin partial-slip closed form, the stick/slip optimality
conditions and the load constraint."""
import numpy as np
import pytest

from oracle import friction as fr
from oracle import operators as ops
from synth import filtered_traction, grid_dict, rough_surface

E, NU = 1.0, 0.3


def test_tangential_compliance_is_the_operators_surface_displacement():
    """C[q] equals the tangential surface displacement of boussinesq_apply
    for a tangential load (odd and even sizes, Nyquist lines included)."""
    for nx, ny, lx, ly in ((16, 12, 1.0, 1.5), (9, 10, 1.0, 1.0)):
        g = grid_dict(nx, ny, 3, lx, ly, 0.2)
        t = filtered_traction(g, seed=nx)
        t[2] = 0.0
        t[:2] -= t[:2].mean(axis=(1, 2), keepdims=True)
        u = ops.boussinesq_apply(g, E, NU, t)['disp'][:2, 0]
        uc = fr.apply_tangential(t[:2], fr.tangential_compliance_symbol(g, E, NU))
        assert np.linalg.norm(u - uc) <= 1e-14 * np.linalg.norm(u)


def _hertz(n, a=0.2, p0=0.01):
    g = grid_dict(n, n, 4, lz=0.25)
    x = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X, Y)
    p = np.where(r < a, p0 * np.sqrt(np.clip(1 - (r / a) ** 2, 0, None)), 0.0)
    return g, r, p


@pytest.mark.parametrize("nu,qy_bound", [(0.0, 1e-12), (0.3, 0.05)])
def test_cattaneo_mindlin_partial_slip(nu, qy_bound):
    """Hertz pressure p0 sqrt(1 - r^2/a^2), Q = Q_x = 0.5 mu P: the stick
    disc has radius c = a (1 - Q / (mu P))^(1/3) and the traction is
    mu p0 [sqrt(1 - r^2/a^2) - (c/a) sqrt(1 - r^2/c^2)] along x (Johnson,
    Contact Mechanics, Sec. 7.2), within the discretisation and periodic
    image error of a = 0.2 L on 128^2 points.  The closed form is exact for
    nu = 0; for nu > 0 it neglects the small slip across x (Johnson notes
    this), so there the transverse traction is only small."""
    n, a, p0, mu = 128, 0.2, 0.01, 0.3
    g, r, p = _hertz(n, a, p0)
    dA = 1.0 / n ** 2
    P = dA * p.sum()
    Q = np.array([0.5 * mu * P, 0.0])
    q, info = fr.tangential_solve(g, E, nu, p, Q, mu, tol=1e-12)
    c = a * (1 - Q[0] / (mu * P)) ** (1 / 3)
    qx = (np.where(r < a, mu * p0 * np.sqrt(np.clip(1 - (r / a) ** 2, 0, None)), 0.0)
          - np.where(r < c, mu * p0 * (c / a) * np.sqrt(np.clip(1 - (r / c) ** 2, 0, None)), 0.0))
    assert np.linalg.norm(q[0] - qx) <= 0.02 * np.linalg.norm(qx)
    assert np.linalg.norm(q[1]) <= qy_bound * np.linalg.norm(qx)
    assert abs(info["stick_fraction"] - (c / a) ** 2) < 0.02
    assert np.allclose(dA * q.sum(axis=(1, 2)), Q, rtol=0, atol=1e-14 * mu * P)


def test_stick_slip_optimality_on_a_rough_pressure():
    """Arbitrary pressure and oblique load: |q| <= mu p everywhere; where
    |q| < mu p the tangential displacement equals one rigid shift; where
    |q| = mu p, u - delta points against q."""
    n, mu = 64, 0.4
    g = grid_dict(n, n, 4, lz=0.25)
    h = rough_surface(n, n, hurst=0.8, k_roll=2, k_cut=16, rms_slope=0.1, seed=3)
    p = np.clip(h - np.quantile(h, 0.8), 0.0, None)
    dA = 1.0 / n ** 2
    W = dA * p.sum()
    Q = np.array([0.3, -0.4]) * mu * W
    q, info = fr.tangential_solve(g, E, NU, p, Q, mu, tol=1e-13)
    C = fr.tangential_compliance_symbol(g, E, NU)
    u = fr.apply_tangential(q, C)
    qa = np.hypot(q[0], q[1])
    rho = mu * p
    assert np.all(qa <= rho * (1 + 1e-12) + 1e-300)
    assert np.allclose(dA * q.sum(axis=(1, 2)), Q, rtol=0, atol=1e-13 * mu * W)
    stick = (rho > 0) & (qa < rho * (1 - 1e-6))
    slip = (rho > 0) & ~stick
    assert stick.any() and slip.any()
    delta = info["delta"]
    scale = np.abs(u).max()
    assert np.max(np.abs(u[:, stick] - delta[:, None])) <= 1e-6 * scale
    s = u[:, slip] - delta[:, None]
    qs = q[:, slip]
    # antiparallel: the tangential component of s along q is <= 0 and the
    # component across q vanishes
    along = np.sum(s * qs, axis=0) / np.hypot(qs[0], qs[1])
    across = (s[0] * qs[1] - s[1] * qs[0]) / np.hypot(qs[0], qs[1])
    assert np.all(along <= 1e-6 * scale)
    assert np.max(np.abs(across)) <= 1e-6 * scale


def test_load_beyond_the_friction_limit_is_rejected():
    g, r, p = _hertz(32)
    W = p.sum() / 32 ** 2
    with pytest.raises(ValueError):
        fr.tangential_solve(g, E, NU, p, np.array([0.31 * W, 0.0]), 0.3)


def test_tangential_compliance_is_symmetric_positive_definite_per_mode():
    """Per nonzero mode the 2x2 compliance is symmetric with eigenvalues
    2 (1 + nu) / (E |k|) times 1 and 1 - nu (along and across n), the
    coupling term vanishing on the Nyquist lines; mode 0 is dropped."""
    g = grid_dict(8, 6, 2, 1.0, 1.5, 0.2)
    C = fr.tangential_compliance_symbol(g, E, NU)
    assert np.array_equal(C[0, 1], C[1, 0])
    assert np.all(C[:, :, 0, 0] == 0.0)
    k1 = np.fft.fftfreq(8, d=1.0 / 8) * 2 * np.pi / 1.0
    k2 = np.fft.fftfreq(6, d=1.0 / 6) * 2 * np.pi / 1.5
    for iy in range(6):
        for ix in range(8):
            if ix == 0 and iy == 0:
                continue
            q = np.hypot(k1[ix], k2[iy])
            f = 2 * (1 + NU) / (E * q)
            ev = np.linalg.eigvalsh(C[:, :, iy, ix])
            if ix == 4 or iy == 3:          # Nyquist: diagonal, entries f (1 - nu n_a^2)
                n1, n2 = k1[ix] / q, k2[iy] / q
                assert np.allclose(sorted(ev), sorted([f * (1 - NU * n1 * n1), f * (1 - NU * n2 * n2)]))
            else:
                assert np.allclose(ev, [f * (1 - NU), f], rtol=1e-14)

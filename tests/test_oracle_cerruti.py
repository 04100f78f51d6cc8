"""Pins of the oracle's coupled normal-tangential contact (CPU only).

The Boussinesq-Cerruti surface response couples the normal and tangential
problems for nu < 1/2 (Sec. 5.1 names friction as an extension of the
contact step; the cross terms are those of the Boussinesq-Cerruti tensor,
eqn B:fourier with the off-diagonal parts of B_00 and B_10).  The pins:
the cross symbol against the pinned operator's surface displacement; the
plane-strain surface strain under a pressure (Hooke's law at a traction-
free-in-shear surface); Maxwell-Betti reciprocity; the full set of contact
and Coulomb conditions of a coupled solution, with every displacement
taken from boussinesq_apply rather than from the contact module's symbols;
the reduction to the uncoupled solve when the cross terms vanish; the
mirror and diagonal symmetries of an axisymmetric indentation."""
import numpy as np
import pytest

from oracle import contact as oc
from oracle import friction as fr
from oracle import operators as ops
from synth import filtered_traction, grid_dict, paraboloid

E, NU = 1.0, 0.3


@pytest.mark.parametrize("nx,ny,lx,ly", [(16, 12, 1.0, 1.5), (9, 10, 1.0, 1.0), (8, 8, 2.0, 1.0)])
def test_surface_response_is_the_operators_surface_displacement(nx, ny, lx, ly):
    """Normal block + tangential block + the two cross blocks reproduce the
    three surface displacement components of boussinesq_apply for a general
    traction (odd and even sizes, Nyquist lines included)."""
    g = grid_dict(nx, ny, 3, lx, ly, 0.2)
    t = filtered_traction(g, seed=nx + ny)
    t -= t.mean(axis=(1, 2), keepdims=True)
    u = ops.boussinesq_apply(g, E, NU, t)['disp'][:, 0]
    K = fr.coupling_symbol(g, E, NU)
    ut = fr.apply_tangential(t[:2], fr.tangential_compliance_symbol(g, E, NU)) + fr.tangential_from_normal(t[2], K)
    u3 = oc.apply_compliance(t[2], oc.surface_compliance_symbol(g, E, NU)) + fr.normal_from_tangential(t[:2], K)
    assert np.linalg.norm(ut - u[:2]) <= 1e-14 * np.linalg.norm(u[:2])
    assert np.linalg.norm(u3 - u[2]) <= 1e-14 * np.linalg.norm(u[2])
    # the cross terms are not negligible here
    assert np.linalg.norm(fr.normal_from_tangential(t[:2], K)) > 0.05 * np.linalg.norm(u[2])


@pytest.mark.parametrize("m", [1, 3])
def test_plane_strain_surface_strain_under_a_pressure(m):
    """p = cos(2 pi m x / L) on the surface: at z = 0 the stresses are
    s11 = s33 = -p (the surface carries no shear) and e22 = 0, so Hooke's law
    gives d u1 / d x1 = -(1 + nu)(1 - 2 nu) p / E, i.e.
    u1 = -(1 + nu)(1 - 2 nu) sin(q x) / (E q), q = 2 pi m / L."""
    n = 16
    g = grid_dict(n, n, 2, lz=0.2)
    x = np.arange(n) / n
    q = 2 * np.pi * m
    p = np.tile(np.cos(q * x), (n, 1))
    ut = fr.tangential_from_normal(p, fr.coupling_symbol(g, E, NU))
    want = -(1 + NU) * (1 - 2 * NU) * np.sin(q * x) / (E * q)
    assert np.max(np.abs(ut[0] - want[None, :])) <= 1e-15
    assert np.max(np.abs(ut[1])) <= 1e-15


def test_maxwell_betti_reciprocity_of_the_cross_terms():
    """The work of a pressure through the normal displacement of a
    tangential traction equals the work of that tangential traction through
    the tangential displacement of the pressure."""
    g = grid_dict(12, 16, 2, 1.0, 0.75, 0.2)
    t = filtered_traction(g, seed=5)
    s = filtered_traction(g, seed=6)
    K = fr.coupling_symbol(g, E, NU)
    w1 = np.sum(s[2] * fr.normal_from_tangential(t[:2], K))
    w2 = np.sum(t[:2] * fr.tangential_from_normal(s[2], K))
    assert abs(w1 - w2) <= 1e-14 * (abs(w1) + abs(w2))
    assert abs(w1) > 0


def _certify(g, h, W, Q, mu, p, q, tol):
    """Normal contact (KKT on h) and Coulomb partial slip for the surface
    traction (q, p), with the surface displacement from boussinesq_apply."""
    n = g['nx'] * g['ny']
    dA = g['lx'] * g['ly'] / n
    t = np.concatenate([q, p[None]], axis=0)
    u = ops.boussinesq_apply(g, E, NU, t)['disp'][:, 0]
    scale = np.max(np.abs(h))
    # normal: p >= 0, gap >= 0, gap = 0 where p > 0, total load
    assert np.all(p >= 0.0)
    c = p > 0
    gap = u[2] - h
    gap -= gap[c].mean()
    assert np.max(np.abs(gap[c])) <= tol * scale
    assert np.min(gap) >= -tol * scale
    assert abs(dA * p.sum() - W) <= 1e-13 * W
    # tangential: |q| <= mu p, one rigid shift on the stick zone, slip
    # against q on the friction limit, total force
    qa = np.hypot(q[0], q[1])
    rho = mu * p
    assert np.all(qa <= rho * (1 + 1e-12) + 1e-300)
    assert np.allclose(dA * q.sum(axis=(1, 2)), Q, rtol=0, atol=1e-13 * mu * W)
    stick = c & (qa < rho * (1 - 1e-6))
    slip = c & ~stick
    assert stick.any() and slip.any()
    ut = u[:2]
    uscale = np.abs(ut[:, c]).max()
    delta = ut[:, stick].mean(axis=1)
    assert np.max(np.abs(ut[:, stick] - delta[:, None])) <= tol * uscale
    sv = ut[:, slip] - delta[:, None]
    qs = q[:, slip]
    along = np.sum(sv * qs, axis=0) / np.hypot(qs[0], qs[1])
    across = (sv[0] * qs[1] - sv[1] * qs[0]) / np.hypot(qs[0], qs[1])
    assert np.all(along <= tol * uscale)
    assert np.max(np.abs(across)) <= tol * uscale
    return u


@pytest.mark.parametrize("Qdir", [(0.4, 0.0), (0.25, -0.3)])
def test_coupled_solution_meets_the_contact_and_coulomb_conditions(Qdir):
    """Paraboloid on 32^2, mu = 0.3, an oblique or axial tangential load: the
    alternation converges and its (p, q) satisfies every contact and
    friction condition with the coupled displacement; the cross terms move
    the solution away from Goodman's by far more than the tolerance."""
    n, mu = 32, 0.3
    g = grid_dict(n, n, 2, lz=0.25)
    h = paraboloid(g, R=0.5)
    W = 2e-3
    Q = np.array(Qdir) * mu * W
    p, q, info = fr.frictional_contact_solve(g, E, NU, h, W, Q, mu, coupled=True, tol=1e-14)
    assert info["change"] < 1e-14 and info["iters"] < 40
    _certify(g, h, W, Q, mu, p, q, 1e-9)
    p0, q0, _ = fr.frictional_contact_solve(g, E, NU, h, W, Q, mu, coupled=False)
    assert np.linalg.norm(q - q0) > 1e-3 * np.linalg.norm(q0)
    assert np.linalg.norm(p - p0) > 1e-4 * np.linalg.norm(p0)


def test_uncoupled_solution_violates_the_coupled_conditions():
    """The Goodman solution is not a solution of the coupled problem: its
    normal gap, computed with the cross terms, is not flat on the contact
    set (so the certificate above can tell the two apart)."""
    n, mu = 32, 0.3
    g = grid_dict(n, n, 2, lz=0.25)
    h = paraboloid(g, R=0.5)
    W = 2e-3
    Q = np.array([0.4, 0.0]) * mu * W
    p0, q0, _ = fr.frictional_contact_solve(g, E, NU, h, W, Q, mu, coupled=False)
    with pytest.raises(AssertionError):
        _certify(g, h, W, Q, mu, p0, q0, 1e-6)


def test_cross_terms_vanish_for_an_incompressible_body():
    """At nu = 1/2 the cross symbol is zero and the coupled alternation
    returns Goodman's solution."""
    n, mu = 32, 0.3
    g = grid_dict(n, n, 2, lz=0.25)
    assert np.all(fr.coupling_symbol(g, E, 0.5) == 0.0)
    h = paraboloid(g, R=0.5)
    W = 2e-3
    Q = np.array([0.3, 0.1]) * mu * W
    p, q, _ = fr.frictional_contact_solve(g, E, 0.5, h, W, Q, mu, coupled=True, tol=1e-14)
    p0, q0, _ = fr.frictional_contact_solve(g, E, 0.5, h, W, Q, mu, coupled=False)
    assert np.linalg.norm(p - p0) <= 1e-12 * np.linalg.norm(p0)
    assert np.linalg.norm(q - q0) <= 1e-10 * np.linalg.norm(q0)


def test_axisymmetric_indentation_without_tangential_load():
    """Q = 0 on a paraboloid centred on a grid node: the pressure pulls the
    surface inwards and friction resists it, so q is nonzero, radial and
    odd about the centre (q1 odd in x, even in y), and the diagonal mirror
    swaps its components; p keeps the indenter's symmetries."""
    n, mu = 32, 0.5
    g = grid_dict(n, n, 2, lz=0.25)
    h = paraboloid(g, R=0.5)
    W = 2e-3
    p, q, info = fr.frictional_contact_solve(g, E, NU, h, W, np.zeros(2), mu, coupled=True, tol=1e-14)
    c = n // 2
    # mirror about the centre node: index i -> 2c - i (mod n)
    mir = (2 * c - np.arange(n)) % n
    assert np.max(np.abs(q)) > 1e-3 * mu * np.max(p)
    assert np.allclose(q[0][:, mir], -q[0], atol=1e-11 * np.max(np.abs(q)))
    assert np.allclose(q[0][mir, :], q[0], atol=1e-11 * np.max(np.abs(q)))
    assert np.allclose(q[1], q[0].T, atol=1e-11 * np.max(np.abs(q)))
    assert np.allclose(p, p.T, atol=1e-12 * np.max(p))
    assert np.allclose(p[:, mir], p, atol=1e-12 * np.max(p))
    # outward on the body: friction opposes the inward surface motion
    X = np.arange(n) - c
    assert np.sum(q[0] * X[None, :]) > 0

"""Pins of the oracle's adhesive contact (Dugdale cohesive zone, CPU only):
the conditions of the solution checked with displacements from the pinned
boussinesq_apply, the exact reductions (no adhesion; a range that covers
the whole surface, whose uniform suction only adds to the load in the
periodic setting), the rigid (Derjaguin) limit of the adhesive force, and
the growth of the contact with the work of adhesion."""
import numpy as np
import pytest

from oracle import adhesion as ad
from oracle import contact as oc
from oracle import operators as ops
from synth import grid_dict, paraboloid, rough_surface

E, NU = 1.0, 0.3


def _certify(g, h, W, sigma0, h0, p, gap, info, tol):
    """p_c >= 0, g >= 0, g = 0 where p_c > 0, C = {g <= h0}, p = p_c -
    sigma0 1_C, dA sum p = W; the gap recomputed from boussinesq_apply's
    surface displacement of the total traction."""
    n = g["nx"] * g["ny"]
    dA = g["lx"] * g["ly"] / n
    pc, C = info["p_c"], info["cohesive"]
    assert np.all(pc >= 0.0)
    assert np.array_equal(p, pc - sigma0 * C)
    assert abs(dA * p.sum() - W) <= 1e-12 * (abs(W) + sigma0 * dA * n)
    t = np.zeros((3,) + h.shape)
    t[2] = p
    u3 = ops.boussinesq_apply(g, E, NU, t)["disp"][2, 0]
    c = pc > 0
    gg = u3 - h
    gg -= gg[c].mean()
    scale = np.max(np.abs(h))
    assert np.max(np.abs(gg - gap)) <= tol * scale
    assert np.max(np.abs(gg[c])) <= tol * scale
    assert np.min(gg) >= -tol * scale
    # the cohesive set is the set of gaps within the range (away from ties)
    assert np.array_equal(C, gap <= h0)
    margin = np.min(np.abs(gap[~c] - h0)) if np.any(~c) else np.inf
    assert margin > 1e3 * tol * scale


@pytest.mark.parametrize("kind", ["paraboloid", "rough"])
def test_solution_meets_the_adhesive_contact_conditions(kind):
    n = 64
    g = grid_dict(n, n, 2, lz=0.25)
    if kind == "paraboloid":
        h = paraboloid(g, R=0.5)
        W, sigma0, h0 = 1e-3, 2e-3, 0.01
    else:
        h = rough_surface(n, n, hurst=0.8, k_roll=2, k_cut=16, rms_slope=0.1, seed=4)
        h = h - h.max()
        W, sigma0, h0 = 5e-4, 5e-3, 2e-3
    p, gap, info = ad.adhesive_contact_solve(g, E, NU, h, W, sigma0, h0)
    assert info["iters"] >= 2 and info["cohesive_fraction"] > info["contact_fraction"] > 0
    _certify(g, h, W, sigma0, h0, p, gap, info, 1e-12)


def test_no_adhesion_is_frictionless_contact():
    n = 32
    g = grid_dict(n, n, 2, lz=0.25)
    h = paraboloid(g, R=0.5)
    p, gap, info = ad.adhesive_contact_solve(g, E, NU, h, 1e-3, 0.0, 0.01)
    p0, gap0, _ = oc.contact_solve(h, 1e-3, g, E, NU, tol=1e-14)
    assert np.max(np.abs(p - p0)) <= 1e-12 * np.max(p0)
    assert np.max(np.abs(gap - gap0)) <= 1e-12 * np.max(np.abs(h))


def test_range_covering_the_surface_only_adds_a_uniform_suction():
    """With h0 above every gap the cohesive set is the whole surface: the
    uniform suction -sigma0 has no mode but the mean, which produces no
    displacement of the periodic half-space, so p_c is the frictionless
    solution under W + sigma0 L^2 and p = p_c - sigma0."""
    n = 32
    g = grid_dict(n, n, 2, lz=0.25)
    h = paraboloid(g, R=0.5)
    sigma0 = 3e-3
    p, gap, info = ad.adhesive_contact_solve(g, E, NU, h, 1e-3, sigma0, 10.0)
    assert np.all(info["cohesive"])
    pc, _, _ = oc.contact_solve(h, 1e-3 + sigma0, g, E, NU, tol=1e-14)
    assert np.max(np.abs(info["p_c"] - pc)) <= 1e-13 * np.max(pc)
    assert np.allclose(p, pc - sigma0, rtol=0, atol=1e-13 * np.max(pc))


def test_rigid_limit_gives_derjaguins_adhesive_force():
    """A very stiff body (E = 1e6) barely deforms: the cohesive set is the
    set of nodes whose profile gap r^2 / (2R) is within h0 of the apex, and
    the adhesive force sigma0 dA |C| approaches Derjaguin's 2 pi R w
    (w = sigma0 h0) up to the lattice count of a disc of radius
    sqrt(2 R h0) = 15 cells."""
    n = 256
    g = grid_dict(n, n, 2, lz=0.25)
    R, sigma0, h0 = 0.5, 2e-3, 3.5e-3
    h = paraboloid(g, R=R)
    p, gap, info = ad.adhesive_contact_solve(g, 1e6, NU, h, 1e-6, sigma0, h0)
    assert np.array_equal(info["cohesive"], -h <= h0 * (1 + 1e-6))
    w = sigma0 * h0
    assert abs(info["adhesive_force"] / (2 * np.pi * R * w) - 1.0) < 0.02


def test_contact_grows_with_the_work_of_adhesion():
    """At a fixed load, a stronger attraction pulls more of the surface
    into contact and into the cohesive zone."""
    n = 128
    g = grid_dict(n, n, 2, lz=0.25)
    h = paraboloid(g, R=0.5)
    areas, forces = [], []
    for sigma0 in (0.0, 2e-3, 5e-3, 1e-2):
        _, _, info = ad.adhesive_contact_solve(g, E, NU, h, 1e-3, sigma0, 0.01)
        areas.append(info["contact_fraction"])
        forces.append(info["adhesive_force"])
    assert all(b >= a for a, b in zip(areas, areas[1:])) and areas[-1] > 1.2 * areas[0], areas
    assert all(b > a for a, b in zip(forces, forces[1:])), forces

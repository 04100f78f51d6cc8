"""Pins of the oracle's Algorithm 1 (Sec. 5.2) on non-flat surfaces, where the
plastic surface displacement U3p feeds back into the contact step (CPU).

A converged elastoplastic contact state (eps_p, e_p, sigma, T, U3p) is the
solution of the coupled problem exactly when these hold, each checked
against quantities the coupling loop does not form itself:

* contact: p = T3 solves the frictionless contact problem on the surface
  modified by the residual displacement, h - U3p (Remark
  rem:modified_contact): p >= 0, dA sum p = W, and the gap is zero on the
  contact set and non-negative elsewhere (KKT certificate);
* bookkeeping of U3p: it equals the surface u3 of N[C : eps_p] for the total
  plastic strain (the steps' increments summed, by linearity);
* equilibrium of the incremental residual summed over the steps: sigma
  equals the stress of the total strain grad_s M[T] + grad_s N[C : eps_p]
  minus C : eps_p (eqn total_strain_n with eqn incremental_strain);
* plastic admissibility and consistency (Sec. 4.1): sigma is inside the
  hardened yield surface everywhere and on it wherever the last step flowed;
* the outer error of Algorithm 1 is below its tolerance.
"""
import os
import sys

import numpy as np
import pytest

from oracle import contact as oc
from oracle import coupling as cp
from oracle import friction as fr
from oracle import operators as ops
from oracle import plasticity as pl
from synth import grid_dict, paraboloid

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
sys.path.insert(0, GOLDEN)
from make_golden import CASES  # noqa: E402


def certificates(g, mat, h, W, st, cerruti=False):
    """The residuals of the list above for a state st (dict of arrays).
    cerruti: the normal surface displacement includes the one of the
    tangential traction (taken from boussinesq_apply)."""
    E, nu = mat["E"], mat["nu"]
    nx, ny = g["nx"], g["ny"]
    p = st["traction"][2]
    Hm = h - st["u3p"]
    if cerruti:
        u = ops.boussinesq_apply(g, E, nu, st["traction"])["disp"][2, 0]
    else:
        u = oc.apply_compliance(p, oc.surface_compliance_symbol(g, E, nu))
    gap = u - Hm
    gap = gap - gap[p > 0].mean()
    dA = g["lx"] * g["ly"] / (nx * ny)
    out = {"kkt": oc.kkt_residual(p, gap, Hm), "neg_p": float(-min(p.min(), 0.0)),
           "load": abs(dA * p.sum() - W) / W}
    r = ops.mindlin_apply(g, E, nu, st["eps_p"])
    out["u3p"] = np.abs(r["surf_u3"] - st["u3p"]).max() / np.abs(st["u3p"]).max()
    f = ops.apply(g, E, nu, eps_p=st["eps_p"], traction=st["traction"])
    out["stress"] = np.abs(f["stress"] - st["sigma"]).max() / np.abs(st["sigma"]).max()
    fy = pl.von_mises(st["sigma"])
    lim = mat["sigma_y0"] + mat["E_h"] * st["ep"]
    out["outside"] = float(max(0.0, (fy - lim).max()) / mat["sigma_y0"])
    return out, fy, lim


def test_algorithm1_fresh_run_certificates_on_a_paraboloid():
    """Two cumulative loads on a paraboloid, 16 x 16 x 4: the second step
    starts from a state with U3p != 0 and T_n != 0."""
    g = grid_dict(16, 16, 4, lz=0.2)
    mat = dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1)
    h = paraboloid(g, R=0.5)
    st = cp.new_state(g)
    tol = 1e-10
    # relax 0.6: same fixed point as the paper's 0.3, half the outer passes
    i1 = cp.elastoplastic_solve(g, mat, h, [0.0005], st, tol_outer=tol, relax=0.6)
    ep1 = st["ep"].copy()
    u3p1 = st["u3p"].copy()
    i2 = cp.elastoplastic_solve(g, mat, h, [0.001], st, tol_outer=tol, relax=0.6)
    for inf in i1 + i2:
        assert inf["outer_err"] < tol
        assert inf["outer_iters"] > 2          # the coupling did iterate
    # the surface feedback is active: U3p is a sizeable part of the profile
    # change over the contact zone and grew in the second step
    assert np.abs(u3p1).max() > 1e-3 * np.abs(h).max()
    assert np.abs(st["u3p"]).max() > np.abs(u3p1).max()
    c, fy, lim = certificates(g, mat, h, 0.001, st)
    assert c["kkt"] < 1e-12, c
    assert c["neg_p"] == 0.0 and c["load"] < 1e-14, c
    assert c["u3p"] < 1e-13, c
    assert c["stress"] < 1e-11, c
    assert c["outside"] < 1e-13, c
    flowed = st["ep"] > ep1
    assert flowed.sum() > 10
    assert np.max(np.abs(fy[flowed] - lim[flowed])) < 1e-12 * mat["sigma_y0"]
    assert 3 <= np.count_nonzero(st["traction"][2]) < 16 * 16 // 2


# KKT bound per stored case: the contact step of the last outer pass sees
# H0 minus the relaxed correction, which differs from h - U3p by about the
# outer tolerance (1e-11 of |H0|_2) -- visible on the rough case, whose
# profile has a small max|h| against its L2 norm; Hertz cases reach 1e-12.
STORED = {"hertz_ep_16x16x8": 1e-12, "rough_ep_16x16x8": 1e-10, "hertz_graded_ep_16x16x8": 1e-12,
          "hertz_friction_ep_16x16x8": 1e-12, "hertz_cerruti_ep_16x16x8": 1e-12, "hertz_adhesion_ep_16x16x8": 1e-12,
          "c1_32x32x16": 1e-12}


def adhesion_certificates(g, mat, h, W, st, sigma0, h0):
    """Dugdale cohesive-zone contact on the surface h - U3p for the stored
    total traction p: with the gap from boussinesq_apply, the cohesive set
    C = {gap <= h0}, p = -sigma0 off contact in C, p = 0 outside C, the
    repulsive part p_c = p + sigma0 1_C >= 0, gap = 0 where p_c > 0 and
    >= 0 everywhere, the load.  The contact set is where p is neither 0 nor
    -sigma0."""
    E, nu = mat["E"], mat["nu"]
    p = st["traction"][2]
    Hm = h - st["u3p"]
    u3 = ops.boussinesq_apply(g, E, nu, st["traction"])["disp"][2, 0]
    tiny = 1e-12 * sigma0
    Ic = (np.abs(p) > tiny) & (np.abs(p + sigma0) > tiny)
    gap = u3 - Hm
    gap -= gap[Ic].mean()
    C = gap <= h0
    pc = p + sigma0 * C
    scale = np.max(np.abs(Hm))
    dA = g["lx"] * g["ly"] / (g["nx"] * g["ny"])
    return {"kkt_on": float(np.max(np.abs(gap[Ic])) / scale), "kkt_off": float(max(0.0, -np.min(gap)) / scale),
            "pc_min": float(np.min(pc) / sigma0), "pc_contact_min": float(np.min(pc[Ic]) / sigma0), "cohesive_off": float(np.max(np.abs(p[C & ~Ic] + sigma0)) / sigma0),
            "outside": float(np.max(np.abs(p[~C])) / sigma0), "load": abs(dA * p.sum() - W) / W,
            "n_contact": int(Ic.sum()), "n_cohesive_off": int((C & ~Ic).sum())}


def friction_certificates(g, mat, W, st, mu_f, q_ratio, cerruti):
    """Coulomb partial slip of the stored tangential traction: |q| <= mu_f p,
    total force q_ratio mu_f W, one rigid shift of the stick zone and slip
    against q on the friction limit, the tangential surface displacement
    taken from boussinesq_apply (of q alone for Goodman's uncoupled form,
    of the whole traction with the Cerruti cross terms)."""
    E, nu = mat["E"], mat["nu"]
    T = np.array(st["traction"])
    if not cerruti:
        T[2] = 0.0
    ut = ops.boussinesq_apply(g, E, nu, T)["disp"][:2, 0]
    q, p = st["traction"][:2], st["traction"][2]
    dA = g["lx"] * g["ly"] / (g["nx"] * g["ny"])
    qa = np.hypot(q[0], q[1])
    rho = mu_f * p
    c = p > 0
    stick = c & (qa < rho * (1 - 1e-6))
    slip = c & ~stick
    scale = np.abs(ut[:, c]).max()
    delta = ut[:, stick].mean(axis=1)
    sv = ut[:, slip] - delta[:, None]
    qs = q[:, slip]
    return {"outside": float(np.max(qa - rho * (1 + 1e-12))),
            "force": float(np.max(np.abs(dA * q.sum(axis=(1, 2)) - np.array(q_ratio) * mu_f * W)) / (mu_f * W)),
            "stick": float(np.max(np.abs(ut[:, stick] - delta[:, None])) / scale),
            "along": float(np.max(np.sum(sv * qs, axis=0) / np.hypot(qs[0], qs[1])) / scale),
            "across": float(np.max(np.abs(sv[0] * qs[1] - sv[1] * qs[0]) / np.hypot(qs[0], qs[1])) / scale),
            "n_stick": int(stick.sum()), "n_slip": int(slip.sum())}


@pytest.mark.parametrize("name", sorted(STORED))
def test_stored_oracle_state_satisfies_the_certificates(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip("stored case %s not written yet" % name)
    d = np.load(path)
    c = CASES[name]
    nx, ny, nz, lz = c["grid"]
    g = grid_dict(nx, ny, nz, lz=lz)
    if "z" in d:
        g["z"] = d["z"]
    steps = int(d["steps_done"]) if "steps_done" in d else len(c["W"])
    st = {k: d[k] for k in ("eps_p", "ep", "sigma", "traction", "u3p")}
    fric = c.get("friction")
    cerruti = bool(fric and fric.get("cerruti"))
    if "adhesion" in c:
        # the normal certificate of adhesive contact replaces the
        # frictionless one
        a = adhesion_certificates(g, c["mat"], d["h"], c["W"][steps - 1], st, *c["adhesion"])
        assert a["kkt_on"] < 1e-12 and a["kkt_off"] < 1e-12, a
        assert a["pc_min"] >= 0 and a["pc_contact_min"] > 0 and a["cohesive_off"] < 1e-12 and a["outside"] < 1e-12 and a["load"] < 1e-12, a
        assert a["n_contact"] > 0 and a["n_cohesive_off"] > 0, a
        cert, fy, lim = certificates(g, c["mat"], d["h"], c["W"][steps - 1], st)
        assert cert["u3p"] < 1e-13 and cert["stress"] < 1e-11 and cert["outside"] < 1e-13, cert
        return
    # with Goodman's friction the normal problem is uncoupled from the
    # tangential one, so the frictionless normal certificate applies; with
    # the Cerruti terms the gap includes the tangential traction's u3
    cert, fy, lim = certificates(g, c["mat"], d["h"], c["W"][steps - 1], st, cerruti=cerruti)
    assert cert["kkt"] < STORED[name], cert
    assert cert["neg_p"] == 0.0 and cert["load"] < 1e-13, cert
    assert cert["u3p"] < 1e-13, cert
    assert cert["stress"] < 1e-11, cert
    assert cert["outside"] < 1e-13, cert
    assert np.count_nonzero(d["ep"]) > 0
    if fric:
        f = friction_certificates(g, c["mat"], c["W"][steps - 1], st, fric["mu_f"], fric["q_ratio"], cerruti)
        assert f["outside"] <= 0.0 and f["force"] < 1e-12, f
        assert f["n_stick"] > 0 and f["n_slip"] > 0, f
        assert f["stick"] < 1e-9 and f["along"] < 1e-9 and f["across"] < 1e-9, f


def test_newton_coupling_reaches_the_algorithm1_fixed_point():
    """Newton-Krylov on Algorithm 1's fixed point (a different iteration)
    ends on Algorithm 1's state and on the certificates of the coupled
    solution, in fewer passes than the relaxed alternation."""
    g = grid_dict(16, 16, 4, lz=0.2)
    mat = dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1)
    h = paraboloid(g, R=0.5)
    Ws = [0.0005, 0.001]
    a = cp.new_state(g)
    ia = cp.elastoplastic_solve(g, mat, h, Ws, a, tol_outer=1e-12, relax=0.6, tol_contact=1e-15)
    b = cp.new_state(g)
    ib = cp.elastoplastic_solve_newton(g, mat, h, Ws, b, tol_outer=1e-13, tol_contact=1e-15)
    for inf in ib:
        assert inf["outer_err"] < 1e-13
    passes_a = sum(i["outer_iters"] for i in ia)
    passes_b = sum(i["evals"] for i in ib)
    assert passes_b < passes_a, (passes_b, passes_a)
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = np.linalg.norm(a[k] - b[k]) / np.linalg.norm(a[k])
        assert err < 1e-9, (k, err)
    c, fy, lim = certificates(g, mat, h, 0.001, b)
    assert c["kkt"] < 1e-12 and c["load"] < 1e-14 and c["u3p"] < 1e-13, c
    assert c["stress"] < 1e-11 and c["outside"] < 1e-13, c

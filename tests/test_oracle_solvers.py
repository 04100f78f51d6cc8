"""Pins of the oracle's return map, contact solver, DF-SANE and Algorithm 1
(CPU only).  Each compares with a closed form, an invariant or an
independent algorithm (dense active-set QP), not with the oracle itself."""
import numpy as np
import pytest

from oracle import contact as oc
from oracle import coupling as cp
from oracle import elastic
from oracle import plasticity as pl
from synth import grid_dict, paraboloid, rough_surface

E, NU = 1.0, 0.3
LAM, MU = elastic.lame(E, NU)
ESTAR = elastic.e_star(E, NU)
SY, EH = 0.01, 0.1


# ------------------------------------------------------------ return map --
def _rand_state(rng, shape, scale):
    d_eps = rng.standard_normal((6,) + shape) * scale
    sig = rng.standard_normal((6,) + shape) * 0.003
    ep = np.abs(rng.standard_normal(shape)) * 0.01
    return d_eps, sig, ep


def test_return_map_yield_consistency_and_flow_direction():
    rng = np.random.default_rng(0)
    d_eps, sig, ep = _rand_state(rng, (200,), 0.004)
    dep, dp, s1 = pl.return_map(d_eps, sig, ep, E, NU, SY, EH)
    flow = dp > 0
    assert 0.2 < flow.mean() < 0.9
    # on the yield surface of the hardened material after the step
    fy = pl.von_mises(s1)
    assert np.max(np.abs(fy[flow] - (SY + EH * (ep + dp))[flow])) < 1e-14 * SY / 1e-2
    # elastic points stay inside, unchanged
    sig_tr = sig + elastic.hooke(d_eps, E, NU)
    assert np.all(pl.von_mises(sig_tr[:, ~flow]) <= SY + EH * ep[~flow] + 1e-16)
    assert np.array_equal(s1[:, ~flow], sig_tr[:, ~flow])
    # deviatoric, coaxial with the trial deviator, equivalent strain = dp
    assert np.max(np.abs(dep[0] + dep[1] + dep[2])) < 1e-17
    st = sig_tr - (sig_tr[0] + sig_tr[1] + sig_tr[2]) / 3.0 * np.array([1, 1, 1, 0, 0, 0])[:, None]
    w = elastic.VOIGT_WEIGHT[:, None]
    cosang = np.sum(w * dep * st, 0)[flow] / np.sqrt(np.sum(w * dep ** 2, 0) * np.sum(w * st ** 2, 0))[flow]
    assert np.max(np.abs(cosang - 1)) < 1e-14
    eq = np.sqrt(2.0 / 3.0 * np.sum(w * dep ** 2, 0))
    assert np.max(np.abs(eq - dp)) < 1e-17


def test_return_map_proportional_path_is_step_independent():
    """Radial return is exact on radial (proportional) deviatoric paths."""
    d = np.zeros((6, 1))
    d[3] = 0.02                      # pure shear strain in the 23 plane
    s0 = np.zeros((6, 1))
    e0 = np.zeros(1)
    a_p, a_d, a_s = pl.return_map(d, s0, e0, E, NU, SY, EH)
    b_p, b_d, b_s = pl.return_map(0.5 * d, s0, e0, E, NU, SY, EH)
    c_p, c_d, c_s = pl.return_map(0.5 * d, b_s, e0 + b_d, E, NU, SY, EH)
    assert abs(a_d[0] - (b_d[0] + c_d[0])) < 1e-17
    assert np.max(np.abs(a_s - c_s)) < 1e-16
    # closed form for pure shear: tau = sqrt(3) (SY + EH ep)/3, 2 mu (g/2 - dp_shear) = tau
    gam = 0.02
    tau_el = 2 * MU * gam
    dp_closed = (np.sqrt(3) * tau_el - SY) / (3 * MU + EH)
    assert abs(a_d[0] - dp_closed) < 1e-16


# --------------------------------------------------------------- contact --
def test_contact_full_contact_sinusoid_exact():
    g = grid_dict(32, 16, 2)
    x = np.arange(32) / 32
    q = 2 * np.pi * 2
    h0 = 1e-3
    h = np.broadcast_to(h0 * np.cos(q * x)[None, :], (16, 32)).copy()
    pbar = 1.2 * ESTAR * q * h0 / 2          # enough for full contact
    p, gap, info = oc.contact_solve(h, pbar, g, E, NU, tol=1e-15, max_iter=200)
    exact = pbar + ESTAR * q * h0 / 2 * np.cos(q * x)[None, :]
    assert np.max(np.abs(p - exact)) < 1e-13 * pbar
    assert info["contact_fraction"] == 1.0


def _dense_compliance(g):
    nx, ny = g['nx'], g['ny']
    n = nx * ny
    sym = oc.surface_compliance_symbol(g, E, NU).ravel()
    jx, jy = np.meshgrid(np.arange(nx), np.arange(ny))
    kx, ky = np.meshgrid(np.arange(nx), np.arange(ny))
    pos = np.stack([jx.ravel() / nx, jy.ravel() / ny], 1)
    kk = np.stack([kx.ravel(), ky.ravel()], 1)
    F = np.exp(-2j * np.pi * pos @ kk.T)         # (points, modes): forward DFT kernel
    # u_i = sum_k sym_k exp(+2 pi i k.x_i) (1/n) sum_j exp(-2 pi i k.x_j) p_j
    return np.real((F.conj() * sym[None, :]) @ F.T) / n


def _active_set_qp(M, h, W, dA):
    """min 1/2 p.Mp - h.p, p >= 0, dA sum p = W, by a primal active-set
    method with exact KKT solves (dense linear algebra)."""
    n = len(h)
    act = np.ones(n, bool)
    for _ in range(10 * n):
        idx = np.where(act)[0]
        m = len(idx)
        K = np.zeros((m + 1, m + 1))
        K[:m, :m] = M[np.ix_(idx, idx)]
        K[:m, m] = -1.0
        K[m, :m] = dA
        rhs = np.concatenate([h[idx], [W]])
        sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
        p = np.zeros(n)
        p[idx] = sol[:m]
        lam = sol[m]
        if np.any(p[idx] < -1e-14 * W):
            worst = idx[np.argmin(p[idx])]
            act[worst] = False
            continue
        p = np.maximum(p, 0)
        g = M @ p - h - lam
        if np.all(g[~act] >= -1e-13 * np.abs(h).max()):
            return p
        add = np.where(~act)[0][np.argmin(g[~act])]
        act[add] = True
    raise RuntimeError("active set did not converge")


def test_contact_matches_dense_active_set_qp():
    g = grid_dict(8, 8, 2)
    h = rough_surface(8, 8, hurst=0.7, k_roll=1, k_cut=3, rms_slope=0.1, seed=3)
    M = _dense_compliance(g)
    dA = 1.0 / 64
    W = 0.002
    ref = _active_set_qp(M, h.ravel(), W, dA).reshape(8, 8)
    p, gap, info = oc.contact_solve(h, W, g, E, NU, tol=1e-15, max_iter=2000)
    assert 0 < info["contact_fraction"] < 1
    assert np.max(np.abs(p - ref)) < 1e-10 * ref.max()


def test_contact_kkt_certificate_rough():
    g = grid_dict(64, 64, 2)
    h = rough_surface(64, 64, hurst=0.8, k_roll=2, k_cut=16, rms_slope=0.1, seed=1)
    W = 0.01
    p, gap, info = oc.contact_solve(h, W, g, E, NU, tol=1e-15, max_iter=5000)
    dA = 1.0 / 64 ** 2
    assert abs(dA * p.sum() - W) < 1e-15 * W * 64
    assert np.all(p >= 0)
    assert info["kkt_residual"] < 1e-11
    assert 0.01 < info["contact_fraction"] < 0.9


def test_contact_from_a_one_point_start_reaches_the_minimiser():
    """Warm start with the whole load on one point far from the contact zone:
    the gap is uniform on that one-point set, the conjugate-gradient step is
    zero, and the overlapping points must still re-enter (with the
    point-load step); the solution is the one from the uniform start and
    passes the KKT certificate."""
    g = grid_dict(16, 16, 2)
    h = paraboloid(g, R=0.5)
    W = 0.002
    ref, _, rinfo = oc.contact_solve(h, W, g, E, NU, tol=1e-15, max_iter=5000)
    p0 = np.zeros((16, 16))
    p0[0, 0] = 1.0
    p, gap, info = oc.contact_solve(h, W, g, E, NU, tol=1e-15, max_iter=5000, p0=p0)
    assert info["kkt_residual"] < 1e-13, info
    assert p[0, 0] == 0.0
    assert np.max(np.abs(p - ref)) < 1e-12 * ref.max()


@pytest.mark.slow
def test_contact_hertz_within_discretisation_error():
    """Paraboloid, a/L ~ 0.1, a/dx ~ 25: Hertz radius and peak pressure."""
    n = 256
    g = grid_dict(n, n, 2)
    R = 1.0
    h = paraboloid(g, R=R)
    a_target = 0.1
    W = 4 * ESTAR * a_target ** 3 / (3 * R)
    p, gap, info = oc.contact_solve(h, W, g, E, NU, tol=1e-12, max_iter=5000)
    p0_hertz = (6 * W * ESTAR ** 2 / (np.pi ** 3 * R ** 2)) ** (1 / 3)
    area = np.count_nonzero(p > 0) / n ** 2
    a_num = np.sqrt(area / np.pi)
    assert abs(p.max() / p0_hertz - 1) < 0.02
    assert abs(a_num / a_target - 1) < 0.02


# --------------------------------------------------------------- DF-SANE --
def test_dfsane_solves_monotone_system():
    rng = np.random.default_rng(4)
    b = rng.standard_normal(50)
    F = lambda x: x + 0.5 * x ** 3 - b + 0.1 * np.roll(x, 1)
    x, Fx, info = cp.dfsane(F, np.zeros(50), lambda a, c: float(a @ c), 1e-13, max_iter=500)
    assert np.linalg.norm(F(x)) < 1e-13
    assert info["iters"] < 200


# --------------------------------------------------- whole chain, closed --
def _uniaxial_closed_form(pbar):
    """Flat surface, uniform pressure: uniaxial strain with J2 + linear hardening.
    Returns eps33 (total), a (plastic eps33), sigma11."""
    if pbar * (1 - 2 * NU) / (1 - NU) <= SY:
        e33 = -pbar / (LAM + 2 * MU)
        return e33, 0.0, LAM * e33
    # (lam+2mu)|e| - 2mu|a| = pbar ;  2mu|e| - 3mu|a| = SY + EH |a|
    A = np.array([[LAM + 2 * MU, -2 * MU], [2 * MU, -(3 * MU + EH)]])
    e, a = np.linalg.solve(A, [pbar, SY])
    return -e, -a, -LAM * e + MU * (-a)


@pytest.mark.parametrize("steps", [1, 3])
def test_flat_surface_uniaxial_strain_closed_form(steps):
    g = grid_dict(8, 8, 4, lz=0.2)
    mat = dict(E=E, nu=NU, sigma_y0=SY, E_h=EH)
    pbar = 0.02
    st = cp.new_state(g)
    Ws = [pbar * (i + 1) / steps for i in range(steps)]
    infos = cp.elastoplastic_solve(g, mat, np.zeros((8, 8)), Ws, st, tol_outer=1e-12)
    e33, a, s11 = _uniaxial_closed_form(pbar)
    assert np.max(np.abs(st['sigma'][2] + pbar)) < 1e-14
    assert np.max(np.abs(st['eps_p'][2] - a)) < 1e-13 * abs(a)
    assert np.max(np.abs(st['eps_p'][0] + a / 2)) < 1e-13 * abs(a)
    assert np.max(np.abs(st['ep'] - abs(a))) < 1e-13 * abs(a)
    assert np.max(np.abs(st['sigma'][0] - s11)) < 1e-13 * abs(s11)
    for inf in infos:
        assert inf["outer_err"] < 1e-12


# ------------------------------------------------- consistent tangent --
def _plastic_points(rng, n):
    """Random states, each at least 5 % away from the yield surface in f."""
    d_eps, sig, ep = _rand_state(rng, (n,), 0.004)
    sig_tr = sig + elastic.hooke(d_eps, E, NU)
    f = pl.von_mises(sig_tr) - (SY + EH * ep)
    keep = np.abs(f) > 0.05 * SY
    return d_eps[:, keep], sig[:, keep], ep[keep], f[keep] > 0


def test_return_map_tangent_matches_central_differences():
    rng = np.random.default_rng(11)
    d_eps, sig, ep, flow = _plastic_points(rng, 400)
    assert 0.2 < flow.mean() < 0.9
    v = rng.standard_normal(d_eps.shape) * 1e-3
    h = 1e-5
    p1, _, _ = pl.return_map(d_eps + h * v, sig, ep, E, NU, SY, EH)
    p0, _, _ = pl.return_map(d_eps - h * v, sig, ep, E, NU, SY, EH)
    fd = (p1 - p0) / (2 * h)
    t = pl.return_map_tangent(d_eps, sig, ep, E, NU, SY, EH, v)
    assert np.all(t[:, ~flow] == 0.0)
    err = np.max(np.abs(t - fd), axis=0)[flow] / np.max(np.abs(fd), axis=0)[flow]
    assert err.max() < 1e-7


def test_return_map_tangent_matches_the_algorithmic_modulus():
    """Closed form of the algorithmic (consistent) tangent modulus of the
    radial return with linear isotropic hardening (Simo and Taylor 1985;
    Simo and Hughes, Computational Inelasticity, Box 3.2): with n the unit
    trial deviator, dg the consistency parameter (|d_eps_p| = dg) and
    theta = 1 - 2 mu dg / |s_tr|, thetab = 1 / (1 + E_h / (3 mu)) - (1 - theta),
    C_alg : v = K tr(v) 1 + 2 mu theta dev(v) - 2 mu thetab n <n, v>.  Since
    sigma = sigma_tr - 2 mu d_eps_p, the tangent of d_eps_p is
    (C : v - C_alg : v) / (2 mu)."""
    rng = np.random.default_rng(12)
    d_eps, sig, ep, flow = _plastic_points(rng, 300)
    d_eps, sig, ep = d_eps[:, flow], sig[:, flow], ep[flow]
    v = rng.standard_normal(d_eps.shape)
    w = elastic.VOIGT_WEIGHT[:, None]
    sig_tr = sig + elastic.hooke(d_eps, E, NU)
    mean = (sig_tr[0] + sig_tr[1] + sig_tr[2]) / 3
    s_tr = sig_tr - mean * np.array([1, 1, 1, 0, 0, 0])[:, None]
    snorm = np.sqrt(np.sum(w * s_tr ** 2, 0))
    n = s_tr / snorm
    dep, dp, _ = pl.return_map(d_eps, sig, ep, E, NU, SY, EH)
    dg = np.sqrt(np.sum(w * dep ** 2, 0))
    theta = 1 - 2 * MU * dg / snorm
    thetab = 1 / (1 + EH / (3 * MU)) - (1 - theta)
    K = LAM + 2 * MU / 3
    trv = v[0] + v[1] + v[2]
    devv = v - trv / 3 * np.array([1, 1, 1, 0, 0, 0])[:, None]
    calg = (K * trv * np.array([1, 1, 1, 0, 0, 0])[:, None] + 2 * MU * theta * devv
            - 2 * MU * thetab * n * np.sum(w * n * v, 0))
    expect = (elastic.hooke(v, E, NU) - calg) / (2 * MU)
    t = pl.return_map_tangent(d_eps, sig, ep, E, NU, SY, EH, v)
    assert np.max(np.abs(t - expect)) < 1e-13 * np.max(np.abs(expect))


def test_newton_krylov_reaches_the_dfsane_root_superlinearly():
    """Newton with the consistent tangent and DF-SANE (different algorithms)
    find the same root; the Newton residuals fall faster than linearly."""
    g = grid_dict(16, 16, 8, lz=0.25)
    mat = dict(E=E, nu=NU, sigma_y0=SY, E_h=EH)
    h = paraboloid(g, R=0.5)
    p, _, _ = oc.contact_solve(h, 0.002, g, E, NU, tol=1e-14)
    dT = np.zeros((3, 16, 16))
    dT[2] = -p
    st = cp.new_state(g)
    a = cp.plasticity(g, mat, dT, st, tol=1e-12, solver="dfsane")
    b = cp.plasticity(g, mat, dT, st, tol=1e-12, solver="newton")
    assert np.count_nonzero(a['d_ep']) > 20
    hist = b['info']['history']
    assert b['info']['iters'] <= 12
    assert hist[-1] < 1e-12 * hist[0] * 10
    # the last reductions outpace the first (superlinear tail)
    assert hist[-1] / hist[-2] < 1e-2
    scale = np.max(np.abs(a['d_eps']))
    assert np.max(np.abs(a['d_eps'] - b['d_eps'])) < 1e-10 * scale
    assert np.max(np.abs(a['d_eps_p'] - b['d_eps_p'])) < 1e-9 * np.max(np.abs(a['d_eps_p']))


def test_newton_system_on_the_plastic_support_is_exact():
    """The Newton step can be found on the plastic support: with J = I - A T
    (A = grad_s N[C : .], T the consistent tangent), solving
    (I - T A) y = -T R and taking delta = -R + A y gives the delta of
    J delta = -R.  Checked with dense matrices built from the oracle's
    operator and tangent on a 4 x 4 x 3 grid (288 unknowns)."""
    from oracle import operators as ops
    g = grid_dict(4, 4, 3, lz=0.2)
    rng = np.random.default_rng(21)
    shape = (6, 3, 4, 4)
    d_eps, sig, ep = _rand_state(rng, shape[1:], 0.004)
    n = int(np.prod(shape))
    _, dp, _ = pl.return_map(d_eps, sig, ep, E, NU, SY, EH)
    assert 0 < np.count_nonzero(dp) < dp.size
    A = np.zeros((n, n))
    T = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        v = e.reshape(shape)
        A[:, k] = ops.mindlin_apply(g, E, NU, v)['strain'].ravel()
        T[:, k] = pl.return_map_tangent(d_eps, sig, ep, E, NU, SY, EH, v).ravel()
    R = rng.standard_normal(n)
    J = np.eye(n) - A @ T
    delta = np.linalg.solve(J, -R)
    y = np.linalg.solve(np.eye(n) - T @ A, -T @ R)
    delta2 = -R + A @ y
    assert np.linalg.norm(delta2 - delta) <= 1e-10 * np.linalg.norm(delta)
    # y lives on the plastic voxels only
    plastic = np.broadcast_to(dp > 0, shape).ravel()
    assert np.all(y[~plastic] == 0.0)

"""GPU parity of the tangential (Coulomb, partial-slip) contact solve with
the FP64 oracle through the C ABI: the same minimiser to the iteration
tolerance, the Cattaneo-Mindlin closed form, the friction limit and load
constraint, and the argument checks."""
import sys

import numpy as np
import pytest
import torch

from oracle import friction as fr
from synth import grid_dict, rough_surface

pytestmark = pytest.mark.gpu

E, NU = 1.0, 0.3


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _rough_pressure(nx, ny, seed, frac=0.8):
    h = rough_surface(nx, ny, hurst=0.8, k_roll=2, k_cut=min(nx, ny) // 4, rms_slope=0.1, seed=seed)
    return np.clip(h - np.quantile(h, frac), 0.0, None)


@pytest.mark.parametrize("nx,ny,lx,ly,mu,qdir", [
    (64, 64, 1.0, 1.0, 0.4, (0.3, -0.4)),
    (128, 64, 2.0, 1.0, 0.3, (0.5, 0.2)),     # nx != ny, lx != ly
    (32, 128, 0.5, 2.0, 0.6, (-0.2, 0.7)),    # long columns
])
def test_tangential_matches_oracle(nx, ny, lx, ly, mu, qdir):
    from paper_1811_11558_amd import Context
    g = grid_dict(nx, ny, 4, lx, ly, 0.25)
    p = _rough_pressure(nx, ny, seed=nx + ny)
    dA = lx * ly / (nx * ny)
    W = dA * p.sum()
    Q = np.array(qdir) * mu * W
    ref, rinfo = fr.tangential_solve(g, E, NU, p, Q, mu, tol=1e-14)
    ctx = Context(g, E, NU)
    q, info = ctx.tangential_solve(torch.from_numpy(p).cuda(), mu, Q, tol=1e-14)
    torch.cuda.synchronize()
    q = q.cpu().numpy()
    err = _rel(q, ref)
    _say(g, "iters gpu/oracle", info["iters"], rinfo["iters"], "err", err, "stick", info["stick_fraction"],
         rinfo["stick_fraction"])
    assert err <= 1e-11
    assert np.all(np.hypot(q[0], q[1]) <= mu * p * (1 + 1e-12) + 1e-300)
    assert np.allclose(dA * q.sum(axis=(1, 2)), Q, rtol=0, atol=1e-12 * mu * W)
    assert abs(info["stick_fraction"] - rinfo["stick_fraction"]) < 0.01
    assert np.allclose(info["shift"], rinfo["delta"], rtol=1e-6, atol=1e-9 * np.abs(rinfo["delta"]).max())
    ctx.close()


def test_tangential_cattaneo_mindlin_nu0():
    """Hertz pressure, Q = 0.5 mu P, nu = 0: the Cattaneo-Mindlin traction
    and stick radius within the discretisation error of 128^2 points."""
    from paper_1811_11558_amd import Context
    n, a, p0, mu = 128, 0.2, 0.01, 0.3
    g = grid_dict(n, n, 4, lz=0.25)
    x = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X, Y)
    p = np.where(r < a, p0 * np.sqrt(np.clip(1 - (r / a) ** 2, 0, None)), 0.0)
    P = p.sum() / n ** 2
    Q = (0.5 * mu * P, 0.0)
    ctx = Context(g, 1.0, 0.0)
    q, info = ctx.tangential_solve(torch.from_numpy(p).cuda(), mu, Q, tol=1e-12)
    q = q.cpu().numpy()
    c = a * (1 - 0.5) ** (1 / 3)
    qx = (np.where(r < a, mu * p0 * np.sqrt(np.clip(1 - (r / a) ** 2, 0, None)), 0.0)
          - np.where(r < c, mu * p0 * (c / a) * np.sqrt(np.clip(1 - (r / c) ** 2, 0, None)), 0.0))
    _say("cattaneo", _rel(q[0], qx), info)
    assert _rel(q[0], qx) <= 0.02
    assert np.linalg.norm(q[1]) <= 1e-10 * np.linalg.norm(qx)
    assert abs(info["stick_fraction"] - (c / a) ** 2) < 0.02
    ctx.close()


def test_tangential_arguments_are_checked():
    from paper_1811_11558_amd import Context, FvimError
    g = grid_dict(32, 32, 4, lz=0.25)
    p = _rough_pressure(32, 32, seed=1)
    W = p.sum() / 32 ** 2
    ctx = Context(g, E, NU)
    pd = torch.from_numpy(p).cuda()
    for mu, Q in ((0.3, (0.31 * W, 0.0)), (0.0, (0.0, 0.0)), (-0.1, (0.0, 0.0)), (0.3, (float("nan"), 0.0))):
        with pytest.raises(FvimError):
            ctx.tangential_solve(pd, mu, Q)
    with pytest.raises(FvimError, match="iteration limit"):
        ctx.tangential_solve(pd, 0.3, (0.2 * W, 0.0), tol=1e-15, max_iter=8)
    # no tangential force: no traction (the minimiser of the energy with
    # zero resultant), from the first check on
    q, info = ctx.tangential_solve(pd, 0.3, (0.0, 0.0))
    assert float(q.abs().max()) == 0.0 and info["iters"] == 8
    ctx.close()


FRICTION_GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.abspath(__file__)),
                                             "golden", "hertz_friction_ep_16x16x8.npz")


@pytest.mark.parametrize("solver", [0, 2])
def test_elastoplastic_with_friction_matches_stored_oracle(solver):
    """Algorithm 1 with Coulomb friction in the contact step (mu_f = 0.3,
    tangential force (0.5, 0.2) mu_f W at each load) on the Hertz case:
    the GPU state (plastic strain, stresses, the three traction components,
    surface correction) reproduces the oracle's stored by
    tests/golden/make_golden.py.  Friction moves the plastic zone (the
    cumulated plastic strain differs from the frictionless case by about
    45 %), so the comparison exercises the tangential traction inside the
    plasticity solves."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(FRICTION_GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = Context(g, 1.0, 0.3, 0.01, 0.1)
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15,
                                              max_plastic=20000, solver=solver, mu_f=0.3, q_ratio=(0.5, 0.2)))
    torch.cuda.synchronize()
    _say([(i["outer_iters"], i["contact_iters"]) for i in infos])
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-11, (k, err)
    ctx.close()


def test_elastoplastic_with_friction_fp32_refined():
    """The same case in the FP32-refined mode with the accelerated outer
    iteration (Anderson 5, warm-started inexact inner solves): within what
    the tolerances allow (1e-8) of the stored float64 oracle state."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(FRICTION_GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = Context(g, 1.0, 0.3, 0.01, 0.1, precision="fp32_refined")
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-12, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15,
                                              max_plastic=20000, anderson_m=5, warm_start=1, inner_rel=0.1,
                                              mu_f=0.3, q_ratio=(0.5, 0.2)))
    torch.cuda.synchronize()
    _say([(i["outer_iters"], i["r_evals"]) for i in infos])
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-8, (k, err)
    ctx.close()


def test_tangential_matches_oracle_at_benchmark_size():
    """256 x 256 (the smallest size of the tangential-contact benchmark; the
    oracle needs about 90 s at 512 x 512), mu_f 0.3, Q = 0.5 mu_f W along x,
    on a seeded rough-surface pressure: the GPU's minimiser is the
    oracle's."""
    from paper_1811_11558_amd import Context
    n = 256
    g = grid_dict(n, n, 2, 1.0, 1.0, 0.25)
    p = _rough_pressure(n, n, seed=7, frac=0.95)
    W = p.sum() / n ** 2
    mu = 0.3
    Q = (0.5 * mu * W, 0.0)
    ref, rinfo = fr.tangential_solve(g, E, NU, p, Q, mu, tol=1e-13)
    ctx = Context(g, E, NU)
    q, info = ctx.tangential_solve(torch.from_numpy(p).cuda(), mu, Q, tol=1e-13)
    torch.cuda.synchronize()
    err = _rel(q.cpu().numpy(), ref)
    _say("256^2 iters gpu/oracle", info["iters"], rinfo["iters"], "err", err)
    assert err <= 1e-11
    ctx.close()

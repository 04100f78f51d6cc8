"""GPU parity of the frictional contact step with the normal and tangential
problems coupled through the Boussinesq-Cerruti cross terms (Sec. 5.1's
friction, eqn B:fourier's off-diagonal terms) against the FP64 oracle,
through the C ABI: the coupled alternation and Goodman's sequence on
paraboloid and rough surfaces (non-square grids and cells, the 256^2
benchmark size), a tangential traction with no tangential load, Algorithm 1
with the coupled contact step against the stored oracle case, and the
argument checks."""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import friction as fr
from synth import grid_dict, paraboloid, rough_surface

pytestmark = pytest.mark.gpu

E, NU = 1.0, 0.3
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "hertz_cerruti_ep_16x16x8.npz")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _case(kind, nx, ny, lx, ly):
    g = grid_dict(nx, ny, 2, lx, ly, 0.25)
    if kind == "paraboloid":
        h = paraboloid(g, R=0.5)
        W = 2e-3 * lx * ly
    else:
        h = rough_surface(nx, ny, hurst=0.8, k_roll=2, k_cut=min(nx, ny) // 4, rms_slope=0.1, seed=nx + ny)
        h = h - h.max()
        W = 1e-3 * lx * ly
    return g, np.ascontiguousarray(h), W


CASES = [
    ("paraboloid", 32, 32, 1.0, 1.0, 0.3, (0.4, 0.0)),
    ("paraboloid", 64, 32, 1.0, 0.5, 0.5, (0.0, 0.0)),        # no tangential load
    ("rough", 64, 32, 1.0, 0.5, 0.4, (0.3, -0.4)),
    ("rough", 128, 64, 2.0, 1.0, 0.3, (-0.2, 0.5)),
    ("rough", 256, 256, 1.0, 1.0, 0.4, (0.3, -0.4)),          # benchmark size
]


@pytest.mark.parametrize("kind,nx,ny,lx,ly,mu,qdir", CASES)
def test_coupled_frictional_contact_matches_oracle(kind, nx, ny, lx, ly, mu, qdir):
    from paper_1811_11558_amd import Context
    g, h, W = _case(kind, nx, ny, lx, ly)
    Q = np.array(qdir) * mu * W
    _say("case", kind, nx, ny, lx, ly, mu, qdir)
    # the entry point runs the normal solves to tol / 10, the tangential
    # ones to tol
    p_ref, q_ref, rinfo = fr.frictional_contact_solve(g, E, NU, h, W, Q, mu, coupled=True, tol=1e-13,
                                                      tol_contact=1e-14, tol_friction=1e-13)
    ctx = Context(g, E, NU)
    t, info = ctx.frictional_contact_solve(torch.from_numpy(h).cuda(), W, mu, Q, coupled=True, tol=1e-13)
    torch.cuda.synchronize()
    t = t.cpu().numpy()
    ep, eq = _rel(t[2], p_ref), _rel(t[:2], q_ref)
    _say("alternations gpu/oracle", info["iters"], rinfo["iters"], "err p", ep, "q", eq,
         "stick", info["stick_fraction"], rinfo["tangential"]["stick_fraction"])
    assert ep <= 1e-11 and eq <= 1e-11
    dA = lx * ly / (nx * ny)
    assert abs(dA * t[2].sum() - W) <= 1e-13 * W
    assert np.all(np.hypot(t[0], t[1]) <= mu * t[2] * (1 + 1e-12) + 1e-300)
    assert np.allclose(dA * t[:2].sum(axis=(1, 2)), Q, rtol=0, atol=1e-12 * mu * W)
    assert info["rel_change"] < 1e-13 and info["iters"] > 2
    assert abs(info["stick_fraction"] - rinfo["tangential"]["stick_fraction"]) < 0.01
    ctx.close()


@pytest.mark.parametrize("kind,nx,ny,lx,ly,mu,qdir", CASES[2:4])
def test_uncoupled_sequence_matches_oracle(kind, nx, ny, lx, ly, mu, qdir):
    """coupled = 0: the frictionless normal solve, then the tangential solve
    under its pressure (Goodman's approximation), as the oracle does."""
    from paper_1811_11558_amd import Context
    g, h, W = _case(kind, nx, ny, lx, ly)
    Q = np.array(qdir) * mu * W
    p_ref, q_ref, _ = fr.frictional_contact_solve(g, E, NU, h, W, Q, mu, coupled=False, tol_contact=1e-14,
                                                  tol_friction=1e-13)
    ctx = Context(g, E, NU)
    t, info = ctx.frictional_contact_solve(torch.from_numpy(h).cuda(), W, mu, Q, coupled=False, tol=1e-13)
    torch.cuda.synchronize()
    t = t.cpu().numpy()
    ep, eq = _rel(t[2], p_ref), _rel(t[:2], q_ref)
    _say("goodman err p", ep, "q", eq)
    assert ep <= 1e-11 and eq <= 1e-11 and info["iters"] == 1
    ctx.close()


def test_warm_start_from_the_solution_stops_at_once():
    """warm = 1 with the converged traction: the first alternation already
    changes nothing beyond the tolerance."""
    from paper_1811_11558_amd import Context
    g, h, W = _case("rough", 64, 32, 1.0, 0.5)
    mu, Q = 0.4, np.array([0.3, -0.4]) * 0.4 * W
    ctx = Context(g, E, NU)
    hd = torch.from_numpy(h).cuda()
    t, info = ctx.frictional_contact_solve(hd, W, mu, Q, tol=1e-13)
    t2, info2 = ctx.frictional_contact_solve(hd, W, mu, Q, tol=1e-13, traction=t.clone(), warm=True)
    torch.cuda.synchronize()
    _say("cold", info["iters"], "warm", info2["iters"])
    assert info2["iters"] <= 2 < info["iters"]
    assert _rel(t2.cpu().numpy(), t.cpu().numpy()) < 1e-12
    ctx.close()


def test_argument_checks():
    from paper_1811_11558_amd import Context, FvimError
    g, h, W = _case("paraboloid", 32, 32, 1.0, 1.0)
    ctx = Context(g, E, NU)
    hd = torch.from_numpy(h).cuda()
    with pytest.raises(FvimError):
        ctx.frictional_contact_solve(hd, W, 0.3, (0.3 * W, 0.0))          # |Q| = mu W: full sliding
    with pytest.raises(FvimError):
        ctx.frictional_contact_solve(hd, W, 0.0, (0.0, 0.0))              # no friction coefficient
    with pytest.raises(FvimError):
        ctx.frictional_contact_solve(hd, -W, 0.3, (0.0, 0.0))
    with pytest.raises(FvimError):
        ctx.frictional_contact_solve(hd, W, 0.3, (0.0, 0.0), tol=0.0)
    ctx.close()


@pytest.mark.parametrize("solver", [0, 2])
def test_elastoplastic_with_coupled_friction_matches_stored_oracle(solver):
    """Algorithm 1 with the coupled contact step (mu_f = 0.3, tangential
    force (0.5, 0.2) mu_f W at each load) on the Hertz case: the GPU state
    reproduces the oracle's stored by tests/golden/make_golden.py, with
    DF-SANE and Newton-Krylov plasticity solves (the outer Newton-Krylov
    coupling on this case is among the stored-fixed-point tests of
    test_gpu_solvers)."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = Context(g, 1.0, 0.3, 0.01, 0.1)
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15,
                                              max_plastic=20000, solver=solver, mu_f=0.3, q_ratio=(0.5, 0.2),
                                              cerruti=1))
    torch.cuda.synchronize()
    _say([(i["outer_iters"], i["contact_iters"]) for i in infos])
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-11, (k, err)
    ctx.close()

"""GPU parity of the adhesive contact step (Dugdale cohesive zone, the
adhesion Sec. 5.1 says the contact step can include) with the FP64 oracle
through the C ABI: the same cohesive set, traction and gap on paraboloid and
rough surfaces up to the 256^2 benchmark size, the frictionless limit,
Algorithm 1 with adhesion against the stored oracle case (DF-SANE,
Newton-Krylov, outer Newton-Krylov), and the argument checks."""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import adhesion as ad
from synth import grid_dict, paraboloid, rough_surface

pytestmark = pytest.mark.gpu

E, NU = 1.0, 0.3
HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "hertz_adhesion_ep_16x16x8.npz")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [
    ("paraboloid", 64, 64, 1.0, 1.0, 1e-3, 2e-3, 0.01),
    ("paraboloid", 128, 64, 2.0, 1.0, 2e-3, 4e-3, 0.005),
    ("rough", 64, 32, 1.0, 0.5, 2.5e-4, 5e-3, 2e-3),
    ("rough", 256, 256, 1.0, 1.0, 5e-4, 5e-3, 2e-3),       # benchmark size
]


def _case(kind, nx, ny, lx, ly):
    g = grid_dict(nx, ny, 2, lx, ly, 0.25)
    if kind == "paraboloid":
        h = paraboloid(g, R=0.5)
    else:
        h = rough_surface(nx, ny, hurst=0.8, k_roll=2, k_cut=min(nx, ny) // 4, rms_slope=0.1, seed=nx + 3 * ny)
        h = h - h.max()
    return g, np.ascontiguousarray(h)


@pytest.mark.parametrize("kind,nx,ny,lx,ly,W,sigma0,h0", CASES)
def test_adhesive_contact_matches_oracle(kind, nx, ny, lx, ly, W, sigma0, h0):
    from paper_1811_11558_amd import Context
    _say("case", kind, nx, ny, lx, ly, W, sigma0, h0)
    g, h = _case(kind, nx, ny, lx, ly)
    p_ref, gap_ref, rinfo = ad.adhesive_contact_solve(g, E, NU, h, W, sigma0, h0, tol=1e-14)
    ctx = Context(g, E, NU)
    p, gap, info = ctx.adhesive_contact_solve(torch.from_numpy(h).cuda(), W, sigma0, h0, tol=1e-14, want_gap=True)
    torch.cuda.synchronize()
    p, gap = p.cpu().numpy(), gap.cpu().numpy()
    C = gap <= h0
    ep, eg = _rel(p, p_ref), np.max(np.abs(gap - gap_ref)) / np.max(np.abs(h))
    _say("set updates gpu/oracle", info["iters"], rinfo["iters"], "err p", ep, "gap", eg,
         "cohesive", int(C.sum()), int(rinfo["cohesive"].sum()), "contact", info["contact_fraction"])
    assert np.array_equal(C, rinfo["cohesive"])
    assert info["iters"] == rinfo["iters"]
    assert ep <= 1e-11 and eg <= 1e-12
    dA = lx * ly / (nx * ny)
    assert abs(dA * p.sum() - W) <= 1e-12 * W
    assert abs(info["adhesive_force"] - rinfo["adhesive_force"]) <= 1e-14 * rinfo["adhesive_force"]
    ctx.close()


def test_no_attraction_is_contact_solve():
    from paper_1811_11558_amd import Context
    g, h = _case("rough", 64, 32, 1.0, 0.5)
    ctx = Context(g, E, NU)
    hd = torch.from_numpy(h).cuda()
    p, _, info = ctx.adhesive_contact_solve(hd, 2.5e-4, 0.0, 1e-3, tol=1e-14)
    p0, _, _ = ctx.contact_solve(hd, 2.5e-4, tol=1e-14)
    torch.cuda.synchronize()
    assert _rel(p.cpu().numpy(), p0.cpu().numpy()) <= 1e-12
    assert info["adhesive_force"] == 0.0
    ctx.close()


def test_argument_checks():
    from paper_1811_11558_amd import Context, EPOptions, FvimError
    g, h = _case("paraboloid", 32, 32, 1.0, 1.0)
    ctx = Context(g, E, NU, 0.01, 0.1)
    hd = torch.from_numpy(h).cuda()
    with pytest.raises(FvimError):
        ctx.adhesive_contact_solve(hd, 1e-3, -1e-3, 0.01)
    with pytest.raises(FvimError):
        ctx.adhesive_contact_solve(hd, 1e-3, 1e-3, -0.01)
    with pytest.raises(FvimError):
        ctx.adhesive_contact_solve(hd, -1.0, 1e-3, 0.01)        # no repulsive load left
    st = ctx.new_state()
    with pytest.raises(FvimError):
        ctx.elastoplastic_solve(hd, [1e-3], st, EPOptions(mu_f=0.3, adhesion=(0.01, 0.003)))
    ctx.close()


@pytest.mark.parametrize("solver,coupling", [(0, 0), (2, 0), (0, 1)])
def test_elastoplastic_with_adhesion_matches_stored_oracle(solver, coupling):
    """Algorithm 1 with the adhesive contact step (sigma0 = 0.01 E, h0 =
    0.003 L) on the Hertz case, with DF-SANE or Newton-Krylov plasticity
    solves and with the outer Newton-Krylov coupling: the state the oracle
    stored (tests/golden/make_golden.py).  The contact solves stop at 1e-14
    (the oracle's 1e-15 lies below the rounding floor of some of the GPU's
    pressure iterations on the modified surfaces)."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = Context(g, 1.0, 0.3, 0.01, 0.1)
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-11 if coupling == 0 else 1e-13, relax=0.3,
                                              tol_plastic=1e-13, tol_contact=1e-14, max_plastic=20000,
                                              solver=solver, coupling=coupling, adhesion=(0.01, 0.003)))
    torch.cuda.synchronize()
    _say([(i["outer_iters"], i["contact_iters"]) for i in infos])
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-11, (k, err)
    ctx.close()

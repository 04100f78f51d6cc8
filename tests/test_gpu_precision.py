"""FP32-refined operator path (float32 transforms, kernel and recurrences;
float64 boundary fields, mean mode, solver vectors, reductions, load
constraint and plastic multiplier) against the FP64 oracle.  Every test
prints the measured error; the bounds are the stated accuracy of this
precision mode."""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import operators as ora
from synth import filtered_eigenstrain, filtered_traction, grid_dict

pytestmark = pytest.mark.gpu
E, NU = 1.0, 0.3
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hertz_ep_16x16x8.npz")

# stated bounds of the FP32-refined mode (relative L2 against the FP64 oracle)
OPERATOR_BOUND = 2e-6
SOLVE_BOUND = 1e-11


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(g, **kw):
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1811_11558_amd import Context
    return Context(g, E, NU, precision="fp32_refined", **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("nx,ny,nz", [(32, 32, 16), (64, 32, 33), (4, 1024, 5), (128, 128, 64)])
def test_fp32_operator_error_vs_oracle(nx, ny, nz):
    g = grid_dict(nx, ny, nz, lz=0.25)
    eps = filtered_eigenstrain(g, seed=nz)
    t = filtered_traction(g, seed=nz + 1)
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t) if nx * ny <= 4096 else None
    ctx = _ctx(g)
    out = ctx.operator_apply(torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda(),
                             want=("strain", "stress", "disp", "surf_u3"))
    torch.cuda.synchronize()
    if ref is None:
        # large grid: sampled modes of the strain against the oracle
        modes = [(0, 0), (0, 1), (1, 0), (64, 64), (5, 17), (100, 3)]
        r = ora.apply(g, E, NU, eps_p=eps, traction=t, modes=modes)["strain_hat"]
        spec = np.fft.fft2(out["strain"].cpu().numpy(), axes=(-2, -1)) / (nx * ny)
        got = np.stack([spec[:, :, ky, kx].T for (ky, kx) in modes])
        err = _rel(got, r)
        _say("fp32 sampled strain", err)
        assert err < OPERATOR_BOUND
        return
    for k in ("strain", "stress", "disp", "surf_u3"):
        err = _rel(out[k].cpu().numpy(), ref[k])
        _say("fp32", nx, ny, nz, k, err)
        assert err < OPERATOR_BOUND, (k, err)


def test_fp32_mean_mode_is_float64():
    """Laterally uniform eigenstrain and traction only excite the mean mode,
    which this mode computes in float64: float64-level agreement."""
    g = grid_dict(16, 16, 9, lz=0.3)
    rng = np.random.default_rng(2)
    prof = rng.standard_normal((6, 9)) * 1e-3
    eps = np.ascontiguousarray(np.broadcast_to(prof[:, :, None, None], (6, 9, 16, 16)))
    t = np.ascontiguousarray(np.broadcast_to((rng.standard_normal(3) * 1e-2)[:, None, None], (3, 16, 16)))
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t)
    ctx = _ctx(g)
    out = ctx.operator_apply(torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda(), want=("strain", "stress"))
    torch.cuda.synchronize()
    for k in ("strain", "stress"):
        err = _rel(out[k].cpu().numpy(), ref[k])
        _say("fp32 mean mode", k, err)
        assert err < 1e-13, (k, err)


def test_fp32_elastoplastic_error_vs_stored_oracle():
    from paper_1811_11558_amd import EPOptions
    ref = np.load(GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = _ctx(g, sigma_y0=0.01, E_h=0.1)
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13,
                                              tol_contact=1e-14))
    torch.cuda.synchronize()
    _say(infos)
    p = st["traction"][2].cpu().numpy()
    area = np.count_nonzero(p > 0)
    area_ref = np.count_nonzero(ref["traction"][2] > 0)
    _say("contact area fp32 / fp64:", area, area_ref)
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say("fp32 solve", k, err)
        assert err < SOLVE_BOUND, (k, err)
    assert area == area_ref

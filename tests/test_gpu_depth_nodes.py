"""GPU parity of the operators on non-uniform depth nodes (Sec. 3.1 leaves
the node spacing free) with the FP64 oracle on the same nodes, through the C
ABI: every depth-pass layout that serves nz, both Nyquist-mode launch forms,
float64 (relative L2 <= 1e-11) and the FP32-refined mode (<= 2e-6), and the
argument checks of the node table."""
import sys

import numpy as np
import pytest
import torch

from oracle import operators as ora
from synth import filtered_eigenstrain, filtered_traction, grid_dict

pytestmark = pytest.mark.gpu

E, NU = 1.0, 0.3
TOL = 1e-11


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def graded_nodes(nz, lz, power=2.0):
    """Nodes refined toward the surface: z_i = lz (i / (nz - 1))^power."""
    z = lz * (np.arange(nz) / (nz - 1)) ** power
    z[-1] = lz
    return z


def _case(nx, ny, nz, lz, seed):
    g = grid_dict(nx, ny, nz, 1.0, 1.0, lz)
    eps = filtered_eigenstrain(g, seed=seed, decay=0.3 * lz)
    t = filtered_traction(g, seed=seed + 1)
    return g, eps, t


@pytest.mark.parametrize("nx,ny,nz,lz,power", [
    (16, 8, 9, 0.3, 2.0),       # 16 lanes x 1 node
    (32, 32, 16, 0.25, 1.5),
    (64, 32, 33, 0.25, 2.0),    # ragged: 32 lanes x 2 nodes and 64 x 1
    (16, 16, 100, 0.5, 2.5),    # 64 lanes x 2 nodes, ragged
    (8, 4, 300, 2.0, 2.0),      # 64 lanes x 8 nodes
    (8, 8, 2, 0.1, 2.0),        # one element
])
def test_non_uniform_nodes_match_oracle_every_layout(nx, ny, nz, lz, power):
    from paper_1811_11558_amd import Context
    g, eps, t = _case(nx, ny, nz, lz, seed=nx + nz)
    z = graded_nodes(nz, lz, power)
    gz = dict(g, z=z)
    _say("case", g, "power", power)
    ref = ora.apply(gz, E, NU, eps_p=eps, traction=t)
    ctx = Context(g, E, NU)
    ctx.set_depth_nodes(z)
    e_d, t_d = torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda()
    ran = 0
    for cfg in [-1] + list(range(8)):        # the default layout, then every explicit one
        try:
            ctx.set_option(ctx.OPT_DEPTH_CONFIG, cfg)
        except Exception:
            continue
        out = ctx.operator_apply(e_d, t_d, want=("strain", "stress", "disp", "surf_u3"))
        torch.cuda.synchronize()
        for k in ("strain", "stress", "disp", "surf_u3"):
            err = _rel(out[k].cpu().numpy(), ref[k])
            assert err <= TOL, (cfg, k, err)
        ran += 1
    assert ran >= 1
    # the Nyquist modes in a launch of their own (side stream) give the same
    ctx.set_option(ctx.OPT_DEPTH_CONFIG, -1)
    ctx.set_option(ctx.OPT_SIDE_STREAM, 1)
    out = ctx.operator_apply(e_d, t_d, want=("strain", "disp"))
    torch.cuda.synchronize()
    for k in ("strain", "disp"):
        assert _rel(out[k].cpu().numpy(), ref[k]) <= TOL, k
    ctx.set_option(ctx.OPT_SIDE_STREAM, 0)
    # back to uniform nodes: the uniform oracle
    ctx.set_depth_nodes(None)
    uni = ora.apply(g, E, NU, eps_p=eps, traction=t)
    out = ctx.operator_apply(e_d, t_d, want=("strain",))
    torch.cuda.synchronize()
    assert _rel(out["strain"].cpu().numpy(), uni["strain"]) <= TOL
    if nz > 2:
        assert _rel(uni["strain"], ref["strain"]) > 1e-4      # the nodes matter
    ctx.close()


def test_non_uniform_nodes_fp32_refined():
    from paper_1811_11558_amd import Context
    g, eps, t = _case(64, 64, 40, 0.4, seed=5)
    z = graded_nodes(40, 0.4, 2.0)
    ref = ora.apply(dict(g, z=z), E, NU, eps_p=eps, traction=t)
    ctx = Context(g, E, NU, precision="fp32_refined")
    ctx.set_depth_nodes(z)
    out = ctx.operator_apply(torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda(),
                             want=("strain", "stress", "surf_u3"))
    torch.cuda.synchronize()
    for k in ("strain", "stress", "surf_u3"):
        err = _rel(out[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err <= 2e-6, (k, err)
    ctx.close()


def test_depth_node_table_is_checked():
    from paper_1811_11558_amd import Context, FvimError, operator_apply_batch
    g = grid_dict(16, 16, 6, lz=0.3)
    ctx = Context(g, E, NU)
    good = graded_nodes(6, 0.3)
    bad = [np.array([0.01, 0.05, 0.1, 0.15, 0.2, 0.3]),       # z[0] != 0
           np.array([0.0, 0.05, 0.05, 0.15, 0.2, 0.3]),       # not increasing
           np.array([0.0, 0.05, 0.1, 0.15, 0.2, 0.31]),       # z[-1] != lz
           np.array([0.0, 0.1, 0.3])]                         # wrong count
    for z in bad:
        with pytest.raises(FvimError):
            ctx.set_depth_nodes(z)
    ctx.set_depth_nodes(good)
    other = Context(g, E, NU)
    eps = torch.from_numpy(filtered_eigenstrain(g, seed=1)).cuda()
    with pytest.raises(FvimError, match="non-uniform"):
        operator_apply_batch([ctx, other], eps_p=[eps, eps])
    ctx.close()
    other.close()


GRADED_GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.abspath(__file__)),
                                           "golden", "hertz_graded_ep_16x16x8.npz")


@pytest.mark.parametrize("solver", [0, 2])
def test_elastoplastic_on_graded_nodes_matches_stored_oracle(solver):
    """Algorithm 1 on the Hertz case with depth nodes z_i = lz (i/7)^2: the
    GPU state reproduces the oracle's (tests/golden/make_golden.py), whose
    scalar products, like the GPU's, use the trapezoid weights of these
    nodes."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(GRADED_GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = Context(g, 1.0, 0.3, 0.01, 0.1)
    ctx.set_depth_nodes(ref["z"])
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15,
                                              max_plastic=20000, solver=solver))
    torch.cuda.synchronize()
    _say([i["outer_iters"] for i in infos])
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-11, (k, err)
    ctx.close()


@pytest.mark.parametrize("precision,tol", [("fp64", TOL), ("fp32_refined", 2e-6)])
def test_graded_nodes_benchmark_size_sampled_modes(precision, tol):
    """256 x 256 x 64 on the graded nodes of the benchmark's --graded 2 run,
    in its launch configuration (tuned layout, streaming loads): the GPU
    output's DFT on sampled modes (k = 0, Nyquist lines, edges, random) is
    the oracle's spectral response on those modes and nodes."""
    from paper_1811_11558_amd import Context
    g = grid_dict(256, 256, 64, 1.0, 1.0, 0.25)
    z = graded_nodes(64, 0.25, 2.0)
    eps = filtered_eigenstrain(g, seed=0)
    t = filtered_traction(g, seed=1000)
    ctx = Context(g, E, NU, precision=precision)
    ctx.set_depth_nodes(z)
    ctx.tune()
    e_d, t_d = torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda()
    ctx.operator_apply(e_d, t_d, want=("strain",))
    out = ctx.operator_apply(e_d, t_d, want=("strain",))
    torch.cuda.synchronize()
    strain = out["strain"].cpu().numpy()
    spec = np.fft.fft2(strain, axes=(-2, -1)) / (256 * 256)
    rng = np.random.default_rng(2)
    modes = [(0, 0), (0, 1), (1, 0), (0, 128), (128, 0), (128, 128), (255, 1), (3, 128), (128, 77)]
    modes += [tuple(int(v) for v in rng.integers(0, 256, 2)) for _ in range(15)]
    ref = ora.apply(dict(g, z=z), E, NU, eps_p=eps, traction=t, modes=modes)["strain_hat"]
    got = np.stack([spec[:, :, ky, kx].T for (ky, kx) in modes])
    err = _rel(got, ref)
    _say(precision, "graded sampled-mode rel err", err, "layout", ctx.get_option(ctx.OPT_DEPTH_CONFIG))
    assert err <= tol, err
    ctx.close()

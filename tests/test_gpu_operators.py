"""GPU parity of the operator path (HIP kernels through the C ABI) against the
FP64 oracle.  Tolerance: relative L2 <= 1e-11 in float64.

Cases span several FFT tiles and lane groups, ragged depth counts (nz not a
multiple of the nodes per lane group), nx != ny, lx != ly, the minimum depth
count, and every lanes-per-mode configuration of the depth kernel.  The
256 x 256 x 64 case is the benchmark workload; there the oracle evaluates a
sample of modes and the GPU output is projected on those modes.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import operators as ora
from oracle import plasticity as opl
from synth import filtered_eigenstrain, filtered_traction, grid_dict

pytestmark = pytest.mark.gpu

E, NU = 1.0, 0.3
TOL = 1e-11


def _ctx(g, **kw):
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1811_11558_amd import Context
    return Context(g, E, NU, **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    (16, 8, 9, 1.0, 0.5, 0.3),       # nx != ny, lx != ly
    (32, 32, 16, 1.0, 1.0, 0.25),    # 16 lanes x 1 node
    (64, 32, 33, 1.0, 1.0, 0.25),    # 32 lanes x 2 nodes, ragged
    (16, 16, 100, 1.0, 1.0, 0.5),    # 64 lanes x 2 nodes, ragged
    (8, 8, 2, 1.0, 1.0, 0.1),        # minimum depth count
    (4, 64, 200, 1.0, 2.0, 1.0),     # 64 lanes x 4 nodes, nx = 4
    (8, 4, 300, 0.5, 1.0, 2.0),      # 64 lanes x 8 nodes
    (4, 1024, 5, 1.0, 4.0, 0.25),    # column kernels with 64 KiB tiles (4 planes per block)
    (4, 2048, 3, 1.0, 8.0, 0.25),    # 128 KiB column tiles
    (8, 4096, 2, 1.0, 8.0, 0.25),    # longest columns (2 planes per block)
    (1024, 4, 3, 4.0, 1.0, 0.25),    # rows of 1024
    (4096, 4, 2, 8.0, 1.0, 0.25),    # longest rows
]


@pytest.mark.parametrize("nx,ny,nz,lx,ly,lz", CASES)
def test_fused_operator_matches_oracle(nx, ny, nz, lx, ly, lz):
    g = grid_dict(nx, ny, nz, lx, ly, lz)
    _say("case", g)
    eps = filtered_eigenstrain(g, seed=nx + ny + nz, decay=0.3 * lz)
    t = filtered_traction(g, seed=7 + nz)
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t)
    ctx = _ctx(g)
    dev = torch.device("cuda")
    out = ctx.operator_apply(torch.from_numpy(eps).to(dev), torch.from_numpy(t).to(dev),
                             want=("strain", "stress", "disp", "surf_u3"))
    torch.cuda.synchronize()
    for k in ("strain", "stress", "disp", "surf_u3"):
        err = _rel(out[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err <= TOL, (k, err)
    ctx.close()


@pytest.mark.parametrize("which", ["mindlin", "boussinesq"])
def test_single_operators_match_oracle(which):
    g = grid_dict(32, 16, 12, 1.0, 1.0, 0.2)
    eps = filtered_eigenstrain(g, seed=3)
    t = filtered_traction(g, seed=4)
    ctx = _ctx(g)
    dev = torch.device("cuda")
    if which == "mindlin":
        ref = ora.mindlin_apply(g, E, NU, eps)
        out = ctx.mindlin_apply(torch.from_numpy(eps).to(dev), want=("strain", "stress", "surf_u3"))
    else:
        ref = ora.boussinesq_apply(g, E, NU, t)
        out = ctx.boussinesq_apply(torch.from_numpy(t).to(dev), want=("strain", "stress", "surf_u3"))
    torch.cuda.synchronize()
    for k in ("strain", "stress", "surf_u3"):
        err = _rel(out[k].cpu().numpy(), ref[k])
        _say(which, k, err)
        assert err <= TOL, (k, err)


def test_k0_exclude_policy():
    g = grid_dict(16, 16, 8, 1.0, 1.0, 0.2)
    t = filtered_traction(g, seed=9) + np.array([0.3, -0.2, 0.5])[:, None, None]
    ref = ora.boussinesq_apply(g, E, NU, t, k0_policy="exclude")
    ctx = _ctx(g, k0="exclude")
    out = ctx.boussinesq_apply(torch.from_numpy(np.ascontiguousarray(t)).cuda(), want=("strain",))
    torch.cuda.synchronize()
    err = _rel(out["strain"].cpu().numpy(), ref["strain"])
    assert err <= TOL, err


def test_benchmark_size_sampled_modes():
    """256 x 256 x 64 in the benchmark's launch configuration (depth layout
    chosen by the tuner, streaming loads): the GPU strain's spectrum against
    the oracle's response on one mode of every group of 4 consecutive modes
    of the mode-major spectrum -- every block of the depth pass, whatever the
    layout, at a random lane group inside it -- plus every Nyquist mode
    (the sign replicas of the main launch) and k = 0: about 8,500 modes."""
    nx = ny = 256
    g = grid_dict(nx, ny, 64, 1.0, 1.0, 0.25)
    eps = filtered_eigenstrain(g, seed=0)
    t = filtered_traction(g, seed=1000)
    ctx = _ctx(g)
    ctx.tune()
    out = ctx.operator_apply(torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda(), want=("strain",))
    torch.cuda.synchronize()
    _say("depth layout", ctx.get_option(ctx.OPT_DEPTH_CONFIG))
    strain = out["strain"].cpu().numpy()
    spec = np.fft.fft2(strain, axes=(-2, -1)) / (nx * ny)
    rng = np.random.default_rng(1)
    kxh = nx // 2 + 1
    nm = kxh * ny                                   # mode-major index m = kx * ny + ky
    picks = 4 * np.arange(nm // 4) + rng.integers(0, 4, nm // 4)
    modes = {(int(m % ny), int(m // ny)) for m in picks}
    modes |= {(ky, nx // 2) for ky in range(ny)} | {(ny // 2, kx) for kx in range(kxh)} | {(0, 0)}
    modes = sorted(modes)
    assert len(modes) > 8000
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t, modes=modes, direct_dft=False)["strain_hat"]  # (M, nz, 6)
    got = np.stack([spec[:, :, ky, kx].T for (ky, kx) in modes])                 # (M, nz, 6)
    err = _rel(got, ref)
    worst = np.abs(got - ref).max() / np.abs(ref).max()
    _say("sampled-mode rel err", err, "modes", len(modes), "max abs err / max abs", worst)
    assert err <= TOL, err
    ctx.close()


def test_benchmark_size_full_field_matches_oracle_fast():
    """256 x 256 x 64 in the benchmark's pinned launch configuration (depth
    layout 64 lanes x 1 node, transform choices (0,4) (1,8) (1,8) (1,8),
    streaming loads): every one of the 4.2M voxels of the fused strain
    against the oracle's fast mode (the same operator with its depth sums
    taken by recurrences; about a minute of CPU)."""
    nx = ny = 256
    g = grid_dict(nx, ny, 64, 1.0, 1.0, 0.25)
    eps = filtered_eigenstrain(g, seed=0, decay=0.1, max_abs=1e-3)
    t = filtered_traction(g, seed=1000, max_abs=1e-2)
    ctx = _ctx(g)
    ctx.set_option(ctx.OPT_DEPTH_CONFIG, 4)
    ctx.set_fft_config([(0, 4), (1, 8), (1, 8), (1, 8)])
    out = ctx.operator_apply(torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda(), want=("strain",))
    torch.cuda.synchronize()
    got = out["strain"].cpu().numpy()
    ctx.close()
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t, sums="recurrence")["strain"]
    err = _rel(got, ref)
    worst = np.abs(got - ref).max() / np.abs(ref).max()
    _say("full-field rel err", err, "max abs err / max abs", worst)
    assert err <= TOL and worst <= TOL, (err, worst)


def test_return_map_matches_oracle():
    g = grid_dict(16, 8, 5)
    rng = np.random.default_rng(12)
    V = (6, 5, 8, 16)
    d_eps = rng.standard_normal(V) * 0.003
    sig = rng.standard_normal(V) * 0.003
    ep = np.abs(rng.standard_normal(V[1:])) * 0.01
    mat = dict(sigma_y0=0.01, E_h=0.1)
    ref = opl.return_map(d_eps, sig, ep, E, NU, mat["sigma_y0"], mat["E_h"])
    ctx = _ctx(g, **mat)
    dev = torch.device("cuda")
    dp, de, sn = ctx.return_map(torch.from_numpy(d_eps).to(dev), torch.from_numpy(sig).to(dev),
                                torch.from_numpy(ep).to(dev))
    torch.cuda.synchronize()
    assert 0.2 < np.mean(ref[1] > 0) < 0.8        # both branches exercised
    for a, b in zip((dp, de, sn), ref):
        assert _rel(a.cpu().numpy(), b) <= 1e-14


def test_operator_is_deterministic():
    g = grid_dict(64, 64, 32)
    eps = torch.from_numpy(filtered_eigenstrain(g, seed=5)).cuda()
    t = torch.from_numpy(filtered_traction(g, seed=6)).cuda()
    ctx = _ctx(g)
    a = ctx.operator_apply(eps, t)["strain"].clone()
    b = ctx.operator_apply(eps, t)["strain"]
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_bad_arguments_raise():
    from paper_1811_11558_amd import FvimError
    g = grid_dict(16, 16, 8)
    ctx = _ctx(g)
    with pytest.raises(FvimError):
        ctx.mindlin_apply(torch.zeros((6, 8, 16, 16), dtype=torch.float32, device="cuda"))
    with pytest.raises(FvimError):
        ctx.mindlin_apply(torch.zeros((6, 8, 16, 15), dtype=torch.float64, device="cuda"))
    with pytest.raises(FvimError):
        ctx.mindlin_apply(torch.zeros((6, 8, 16, 16), dtype=torch.float64))


@pytest.mark.parametrize("nz", [16, 33, 64, 100])
def test_every_depth_layout_matches_oracle(nz):
    """Each thread layout of the depth pass that serves nz gives the oracle's
    result (and the tuner picks one of them)."""
    g = grid_dict(16, 8, nz, 1.0, 1.0, 0.3)
    eps = filtered_eigenstrain(g, seed=nz)
    t = filtered_traction(g, seed=nz + 1)
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t)
    ctx = _ctx(g)
    e_d, t_d = torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda()
    ran = 0
    for cfg in range(8):
        try:
            ctx.set_option(ctx.OPT_DEPTH_CONFIG, cfg)
        except Exception:
            continue
        out = ctx.operator_apply(e_d, t_d, want=("strain", "disp"))
        torch.cuda.synchronize()
        for k in ("strain", "disp"):
            err = _rel(out[k].cpu().numpy(), ref[k])
            assert err <= TOL, (cfg, k, err)
        ran += 1
    assert ran >= 1
    ctx.tune()
    ctx.operator_apply(e_d, t_d)
    torch.cuda.synchronize()
    assert 0 <= ctx.get_option(ctx.OPT_DEPTH_CONFIG) < 8


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_nyquist_replicas_in_main_launch_equal_separate_launch(precision):
    """The default launch evaluates each Nyquist mode's sign replicas as
    modes of the main depth launch and averages them afterwards; with the
    side stream on, a launch of its own sums them in turn.  Both give the
    oracle's result, and agree with each other to rounding, on every output
    (stress and displacement included) and on a grid with the corner mode."""
    g = grid_dict(32, 16, 12, 1.0, 0.5, 0.3)
    eps = filtered_eigenstrain(g, seed=7)
    t = filtered_traction(g, seed=8)
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t)
    ctx = _ctx(g, precision=precision)
    e_d, t_d = torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda()
    want = ("strain", "stress", "disp", "surf_u3")
    outs = {}
    for side in (0, 1):
        ctx.set_option(ctx.OPT_SIDE_STREAM, side)
        outs[side] = {k: v.cpu().numpy() for k, v in ctx.operator_apply(e_d, t_d, want=want).items()}
        torch.cuda.synchronize()
    tol = TOL if precision == "fp64" else 2e-6
    for k in want:
        for side in (0, 1):
            err = _rel(outs[side][k], ref[k])
            assert err <= tol, (side, k, err)
        d = _rel(outs[0][k], outs[1][k])
        _say(precision, k, "replicas in main launch vs separate launch", d)
        assert d <= (1e-14 if precision == "fp64" else 1e-6), (k, d)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_streaming_loads_do_not_change_results(precision):
    """Streaming (non-temporal) loads change only how the transforms read
    their input: every output is bitwise the same with them forced on and
    off, and matches the oracle."""
    g = grid_dict(64, 32, 10, 1.0, 0.5, 0.3)
    eps = filtered_eigenstrain(g, seed=11)
    t = filtered_traction(g, seed=12)
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t)
    ctx = _ctx(g, precision=precision)
    e_d, t_d = torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda()
    want = ("strain", "stress", "disp", "surf_u3")
    outs = {}
    for mode in (0, 1):
        ctx.set_option(ctx.OPT_STREAMING, mode)
        outs[mode] = {k: v.cpu().numpy() for k, v in ctx.operator_apply(e_d, t_d, want=want).items()}
        torch.cuda.synchronize()
    tol = TOL if precision == "fp64" else 2e-6
    for k in want:
        assert np.array_equal(outs[0][k], outs[1][k]), k
        assert _rel(outs[1][k], ref[k]) <= tol, k


BATCH = [(16, 16, 9, 1.0, 1.0, 0.3), (32, 16, 16, 1.0, 0.5, 0.25), (64, 64, 33, 1.0, 1.0, 0.25),
         (8, 32, 5, 0.5, 1.0, 0.2)]


def test_batched_operator_uneven_grids():
    """Four grids of different sizes in one batched application (their
    transforms in shared launches): each result matches the oracle and the
    context's own application (the batch uses one depth layout for all, so
    only the order of the depth sums can differ)."""
    from paper_1811_11558_amd import operator_apply_batch
    dev = torch.device("cuda")
    ctxs, eps, ts, refs, own = [], [], [], [], []
    for (nx, ny, nz, lx, ly, lz) in BATCH:
        g = grid_dict(nx, ny, nz, lx, ly, lz)
        e = filtered_eigenstrain(g, seed=nx + 3 * ny + nz, decay=0.3 * lz)
        t = filtered_traction(g, seed=11 + nz)
        refs.append(ora.apply(g, E, NU, eps_p=e, traction=t))
        c = _ctx(g)
        ctxs.append(c)
        eps.append(torch.from_numpy(e).to(dev))
        ts.append(torch.from_numpy(t).to(dev))
        own.append(c.operator_apply(eps[-1], ts[-1], want=("strain", "surf_u3")))
    got = operator_apply_batch(ctxs, eps, ts, want=("strain", "surf_u3"))
    torch.cuda.synchronize()
    for i, (r, o, gb) in enumerate(zip(refs, own, got)):
        for k in ("strain", "surf_u3"):
            e_or = _rel(gb[k].cpu().numpy(), r[k])
            e_own = _rel(gb[k].cpu().numpy(), o[k].cpu().numpy())
            _say("batch", BATCH[i][:3], k, e_or, e_own)
            assert e_or <= TOL and e_own <= 1e-13, (i, k, e_or, e_own)
    for c in ctxs:
        c.close()


def test_persistent_batched_operator_equals_batched_launches():
    """The persistent batched operator (FVIM_OPT_PERSISTENT: every stage in
    one cooperative launch, blocks looping over each stage with a grid
    barrier between stages) on eight grids of different sizes, nz from 8
    to 64: bitwise the multi-launch batched application, which matches the
    oracle."""
    from paper_1811_11558_amd import Context, operator_apply_batch
    dev = torch.device("cuda")
    shapes = [(64, 64, 32), (32, 32, 16), (128, 128, 64), (64, 32, 16), (32, 64, 32), (64, 64, 16),
              (128, 64, 32), (32, 32, 8)]
    ctxs, eps, ts = [], [], []
    for i, (nx, ny, nz) in enumerate(shapes):
        g = grid_dict(nx, ny, nz, 1.0, 1.0, 0.25)
        ctxs.append(Context(g, E, NU))
        eps.append(torch.from_numpy(filtered_eigenstrain(g, seed=i)).to(dev))
        ts.append(torch.from_numpy(filtered_traction(g, seed=1000 + i)).to(dev))
    multi = [o["strain"].clone() for o in operator_apply_batch(ctxs, eps, ts)]
    ctxs[0].set_option(ctxs[0].OPT_PERSISTENT, 1)
    for rep in range(2):             # the second call reuses the table buffer
        pers = operator_apply_batch(ctxs, eps, ts)
        torch.cuda.synchronize()
        for i, (m, p) in enumerate(zip(multi, pers)):
            assert torch.equal(m, p["strain"]), (rep, shapes[i])
    g = grid_dict(*shapes[7], 1.0, 1.0, 0.25)
    ref = ora.apply(g, E, NU, eps_p=eps[7].cpu().numpy(), traction=ts[7].cpu().numpy())["strain"]
    assert _rel(pers[7]["strain"].cpu().numpy(), ref) <= TOL
    # a batch that does not qualify (stress requested) takes the launches
    out = operator_apply_batch(ctxs[:2], eps[:2], ts[:2], want=("strain", "stress"))
    torch.cuda.synchronize()
    assert torch.equal(out[0]["strain"], multi[0])
    for c in ctxs:
        c.close()


def test_batched_operator_more_than_eight_contexts_and_fp32():
    """Eleven contexts (two depth launches of at most eight grids each) in
    float64, and the same grids in the FP32-refined precision against their
    own float32 applications."""
    from paper_1811_11558_amd import Context, operator_apply_batch
    dev = torch.device("cuda")
    for prec, bound in (("fp64", 1e-13), ("fp32_refined", 1e-6)):
        ctxs, eps, own = [], [], []
        for i in range(11):
            g = grid_dict(8 << (i % 3), 8 << ((i // 3) % 2), 3 + i, 1.0, 1.0, 0.25)
            e = torch.from_numpy(filtered_eigenstrain(g, seed=100 + i)).to(dev)
            c = Context(g, E, NU, precision=prec)
            ctxs.append(c)
            eps.append(e)
            own.append(c.operator_apply(e, None, want=("strain",))["strain"])
        got = operator_apply_batch(ctxs, eps, None, want=("strain",))
        torch.cuda.synchronize()
        worst = max(_rel(gb["strain"].cpu().numpy(), o.cpu().numpy()) for gb, o in zip(got, own))
        _say("batch of 11", prec, worst)
        assert worst <= bound
        for c in ctxs:
            c.close()


def _sampled_dft_gpu(f, modes):
    """Fourier coefficients (1/(nx ny)) sum_x f(x) exp(-2 pi i (kx x/nx +
    ky y/ny)) of a real device tensor (..., ny, nx) at the (ky, kx) bins,
    evaluated on the device by matrix products (test-side measurement)."""
    ny, nx = f.shape[-2:]
    dev = f.device
    kx = torch.tensor([m[1] for m in modes], dtype=torch.int64, device=dev)
    ky = torch.tensor([m[0] for m in modes], dtype=torch.int64, device=dev)
    ax = (2 * np.pi / nx) * ((kx[:, None] * torch.arange(nx, device=dev)[None, :]) % nx).double()
    ay = (2 * np.pi / ny) * ((ky[:, None] * torch.arange(ny, device=dev)[None, :]) % ny).double()
    F = f.reshape(-1, nx)
    xr = (F @ torch.cos(ax).T).reshape(-1, ny, len(modes))
    xi = -(F @ torch.sin(ax).T).reshape(-1, ny, len(modes))
    cy, sy = torch.cos(ay).T, torch.sin(ay).T
    re = (xr * cy).sum(1) + (xi * sy).sum(1)
    im = (xi * cy).sum(1) - (xr * sy).sum(1)
    out = torch.complex(re, im) / (nx * ny)
    return out.reshape(tuple(f.shape[:-2]) + (len(modes),)).cpu().numpy()


@pytest.mark.parametrize("nx,ny,nz,prec,bound", [(1024, 1024, 64, "fp64", TOL),
                                                 (512, 512, 128, "fp32_refined", 2e-6)])
def test_full_size_sampled_modes(nx, ny, nz, prec, bound):
    """The rough-contact grid 1024^2 x 64 in float64 and the mixed-precision
    grid 512^2 x 128 in FP32_REFINED, at the launch configuration of the
    benchmark: the strain's Fourier coefficients on sampled bins (k = 0,
    Nyquist lines and corner, edges, random) against the oracle's response on
    those bins.  Eigenstrain in four layers (the others zero) plus traction."""
    from paper_1811_11558_amd import Context
    g = grid_dict(nx, ny, nz, 1.0, 1.0, 0.25)
    eps = filtered_eigenstrain(g, seed=7, layers=[0, 1, nz // 2, nz - 1])
    t = filtered_traction(g, seed=1001)
    rng = np.random.default_rng(2)
    modes = [(0, 0), (0, 1), (1, 0), (0, nx // 2), (ny // 2, 0), (ny // 2, nx // 2), (ny - 1, 1),
             (3, nx // 2), (ny // 2, 77)]
    modes += [(int(rng.integers(0, ny)), int(rng.integers(0, nx))) for _ in range(15)]
    ref = ora.apply(g, E, NU, eps_p=eps, traction=t, modes=modes)["strain_hat"]     # (M, nz, 6)
    ctx = Context(g, E, NU, precision=prec)
    _say("case", nx, ny, nz, prec)
    out = ctx.operator_apply(torch.from_numpy(eps).cuda(), torch.from_numpy(t).cuda(), want=("strain",))
    torch.cuda.synchronize()
    got = np.transpose(_sampled_dft_gpu(out["strain"], modes), (2, 1, 0))          # (M, nz, 6)
    err = _rel(got, ref)
    _say("full-size sampled-mode rel err", nx, ny, nz, prec, err)
    assert err <= bound, err
    ctx.close()


FFT_GRIDS = [(32, 64, 6, 1.0, 1.0, 0.25), (256, 128, 4, 1.0, 0.5, 0.2), (1024, 32, 3, 2.0, 1.0, 0.25),
             (64, 1024, 3, 1.0, 2.0, 0.25), (512, 512, 2, 1.0, 1.0, 0.25)]
FFT_CHOICES = [(t, r) for r in (4, 8) for t in (0, 1, 2)]


@pytest.mark.parametrize("nx,ny,nz,lx,ly,lz", FFT_GRIDS)
def test_every_fft_choice_matches_oracle(nx, ny, nz, lx, ly, lz):
    """Every launch choice of the four transform kernels (half, default and
    double LDS tile; radix-4 and radix-8 stages), uniform and mixed, gives
    the oracle's fields (float64 to 1e-11, float32 to 2e-6) on grids whose
    lengths span the tunable range 32 .. 1024."""
    g = grid_dict(nx, ny, nz, lx, ly, lz)
    e = filtered_eigenstrain(g, seed=nx + ny, decay=0.5 * lz)
    t = filtered_traction(g, seed=nz + 5)
    ref = ora.apply(g, E, NU, eps_p=e, traction=t)
    dev = torch.device("cuda")
    ed, td = torch.from_numpy(e).to(dev), torch.from_numpy(t).to(dev)
    cfgs = [[ch] * 4 for ch in FFT_CHOICES] + [[(0, 8), (2, 4), (1, 8), (2, 8)], [(2, 8), (0, 8), (0, 4), (1, 8)]]
    for prec, bound in (("fp64", TOL), ("fp32_refined", 2e-6)):
        c = _ctx(g, precision=prec)
        for cfg in cfgs:
            c.set_fft_config(cfg)
            out = c.operator_apply(ed, td, want=("strain", "surf_u3"))
            torch.cuda.synchronize()
            errs = [_rel(out[k].cpu().numpy(), ref[k]) for k in ("strain", "surf_u3")]
            _say("fft choice", (nx, ny, nz), prec, cfg, errs)
            assert max(errs) <= bound, (cfg, errs)
        c.close()


def test_fft_tuner_picks_and_records_a_choice():
    """FVIM_OPT_TUNE times the transform choices on the call's own data: the
    result matches the oracle, and a second context of the same shape that
    asks for tuning takes the recorded choices (and depth layout) and gives
    bitwise the same fields."""
    g = grid_dict(256, 128, 8, 1.0, 1.0, 0.25)
    e = filtered_eigenstrain(g, seed=3)
    t = filtered_traction(g, seed=4)
    ref = ora.apply(g, E, NU, eps_p=e, traction=t)
    dev = torch.device("cuda")
    ed, td = torch.from_numpy(e).to(dev), torch.from_numpy(t).to(dev)
    c1 = _ctx(g)
    c1.tune()
    o1 = c1.operator_apply(ed, td, want=("strain",))["strain"]
    cfg1, d1 = c1.fft_config(), c1.get_option(c1.OPT_DEPTH_CONFIG)
    c2 = _ctx(g)
    c2.tune()
    o2 = c2.operator_apply(ed, td, want=("strain",))["strain"]
    torch.cuda.synchronize()
    _say("tuned", cfg1, d1)
    assert c2.fft_config() == cfg1 and c2.get_option(c2.OPT_DEPTH_CONFIG) == d1
    assert all(t_ in (0, 1, 2) and r in (4, 8) for t_, r in cfg1)
    assert torch.equal(o1, o2)
    assert _rel(o1.cpu().numpy(), ref["strain"]) <= TOL
    c1.close()
    c2.close()


def test_batched_transforms_same_alone_and_in_a_batch():
    """Eight small grids of different sizes share one launch per transform
    stage, a ninth grid (1024 x 16) keeps its own transform launches: every
    grid's fields are bitwise those of the same grid batched alone, and
    match the oracle."""
    from paper_1811_11558_amd import operator_apply_batch
    dev = torch.device("cuda")
    shapes = [(64, 64, 12), (32, 32, 8), (128, 128, 6), (64, 32, 8), (32, 64, 10), (64, 64, 4), (128, 64, 6),
              (16, 16, 5), (1024, 16, 3)]
    ctxs, eps, ts, refs = [], [], [], []
    for i, (nx, ny, nz) in enumerate(shapes):
        g = grid_dict(nx, ny, nz, 1.0, 1.0, 0.25)
        e = filtered_eigenstrain(g, seed=40 + i)
        t = filtered_traction(g, seed=60 + i)
        refs.append(ora.apply(g, E, NU, eps_p=e, traction=t))
        ctxs.append(_ctx(g))
        eps.append(torch.from_numpy(e).to(dev))
        ts.append(torch.from_numpy(t).to(dev))
    got = operator_apply_batch(ctxs, eps, ts, want=("strain", "surf_u3"))
    torch.cuda.synchronize()
    for i in range(len(shapes)):
        alone = operator_apply_batch([ctxs[i]], [eps[i]], [ts[i]], want=("strain", "surf_u3"))[0]
        torch.cuda.synchronize()
        for k in ("strain", "surf_u3"):
            err = _rel(got[i][k].cpu().numpy(), refs[i][k])
            _say("batched", shapes[i], k, err)
            assert err <= TOL, (shapes[i], k, err)
            assert torch.equal(got[i][k], alone[k]), (shapes[i], k)
    for c in ctxs:
        c.close()

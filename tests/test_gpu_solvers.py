"""GPU parity of the solvers (contact, plasticity fixed point, Algorithm 1)
with the FP64 oracle, through the C ABI.

Both sides iterate to tight tolerances; iterates are not compared step by
step (the iterations differ in rounding), the converged results are, to the
stated bound.  Where the result has a closed form (flat surface, uniaxial
strain) it is checked as well."""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import contact as oc
from oracle import elastic
from synth import grid_dict, rough_surface

pytestmark = pytest.mark.gpu

E, NU, SY, EH = 1.0, 0.3, 0.01, 0.1
LAM, MU = elastic.lame(E, NU)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx(g, **kw):
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1811_11558_amd import Context
    return Context(g, E, NU, SY, EH, **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n,W,seed", [(32, 0.004, 1), (64, 0.01, 2), (128, 0.02, 3)])
def test_contact_matches_oracle(n, W, seed):
    g = grid_dict(n, n, 2)
    h = rough_surface(n, n, hurst=0.8, k_roll=2, k_cut=n // 4, rms_slope=0.1, seed=seed)
    ref, rgap, rinfo = oc.contact_solve(h, W, g, E, NU, tol=1e-15, max_iter=20000)
    ctx = _ctx(g)
    p, gap, info = ctx.contact_solve(torch.from_numpy(h).cuda(), W, tol=1e-15, max_iter=20000, want_gap=True)
    torch.cuda.synchronize()
    p = p.cpu().numpy()
    err = _rel(p, ref)
    _say("contact", n, "iters gpu/oracle", info["iters"], rinfo["iters"], "rel err", err,
         "frac", info["contact_fraction"])
    assert err < 1e-11
    assert np.all(p >= 0)
    assert abs(p.sum() / n ** 2 - W) < 1e-14 * W * n
    gap = gap.cpu().numpy()
    assert oc.kkt_residual(p, gap, h) < 1e-10
    # the certificate the C ABI reports is formed on the device from the same
    # final gap: the oracle's definition applied to the returned p and gap
    kkt = oc.kkt_residual(p, gap, h)
    assert abs(info["kkt_residual"] - kkt) <= 1e-12 * max(kkt, 1e-300), (info["kkt_residual"], kkt)


def test_contact_matches_oracle_rough_1024():
    """The rough-surface workload's contact solve at its full size: 1024^2,
    Hurst 0.8, PSD plateau for 1 <= |k| < 4, cut-off |k| = 256, rms slope
    0.1, first of 5 load increments to W = 1e-4 (W = 2e-5).  The oracle's
    Polonsky-Keer solve (13 s on 4 host cores) against the GPU's, both to
    tol 1e-15: pressures to 1e-11, identical contact sets, KKT below 1e-12."""
    n, W = 1024, 2e-5
    g = grid_dict(n, n, 64, lz=0.25)
    h = rough_surface(n, n, hurst=0.8, k_roll=4, k_cut=256, rms_slope=0.1, seed=0)
    _say("contact 1024^2: oracle")
    ref, rgap, rinfo = oc.contact_solve(h, W, g, E, NU, tol=1e-15, max_iter=20000)
    ctx = _ctx(g)
    p, gap, info = ctx.contact_solve(torch.from_numpy(h).cuda(), W, tol=1e-15, max_iter=20000, want_gap=True)
    torch.cuda.synchronize()
    p = p.cpu().numpy()
    err = _rel(p, ref)
    _say("contact 1024^2 iters gpu/oracle", info["iters"], rinfo["iters"], "rel err", err, "frac",
         info["contact_fraction"], "kkt", info["kkt_residual"])
    assert err < 1e-11
    assert np.array_equal(p > 0, ref > 0)
    assert abs(p.sum() / n ** 2 - W) < 1e-14 * W * n
    assert info["kkt_residual"] < 1e-12
    kkt = oc.kkt_residual(p, gap.cpu().numpy(), h)
    assert abs(info["kkt_residual"] - kkt) <= 1e-12 * max(kkt, 1e-300)
    ctx.close()


def test_contact_from_a_one_point_start_reaches_the_minimiser():
    """A warm start with the whole load on one point far from the contact
    zone (zero conjugate-gradient step on a one-point contact set): the GPU
    still re-admits the overlapping points and ends on the oracle's
    minimiser from the uniform start."""
    from synth import paraboloid
    g = grid_dict(16, 16, 2)
    h = paraboloid(g, R=0.5)
    W = 0.002
    ref, _, _ = oc.contact_solve(h, W, g, E, NU, tol=1e-15, max_iter=5000)
    p0 = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    p0[0, 0] = 1.0
    p, gap, info = _ctx(g).contact_solve(torch.from_numpy(h).cuda(), W, tol=1e-15, max_iter=5000, p=p0,
                                         want_gap=True)
    torch.cuda.synchronize()
    p = p.cpu().numpy()
    _say("one-point start: iters", info["iters"], "kkt", info["kkt_residual"])
    assert info["kkt_residual"] < 1e-13
    assert _rel(p, ref) < 1e-11


def test_contact_solve_on_workspace_that_held_nan():
    """The solver workspace of a new context is not cleared memory: pages
    that held NaN are freed first, then a contact solve on
    a fresh context (which allocates its workspace then) must stay finite
    and equal a solve on an ordinary context.  The conjugate direction of the
    first iteration must not be formed from what the array held."""
    n, W = 64, 0.01
    g = grid_dict(n, n, 2)
    h = torch.from_numpy(rough_surface(n, n, hurst=0.8, k_roll=2, k_cut=n // 4, rms_slope=0.1, seed=2)).cuda()
    ref, _, _ = _ctx(g).contact_solve(h, W, tol=1e-14, max_iter=20000)
    torch.cuda.synchronize()
    junk = torch.full((1 << 26,), float("nan"), dtype=torch.float64, device="cuda")   # 512 MiB
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    p, _, info = _ctx(g).contact_solve(h, W, tol=1e-14, max_iter=20000)
    torch.cuda.synchronize()
    _say("contact after NaN pages: iters", info["iters"])
    assert torch.isfinite(p).all()
    assert torch.equal(p, ref)


def test_contact_full_contact_sinusoid_exact():
    g = grid_dict(32, 16, 2)
    x = np.arange(32) / 32
    q = 2 * np.pi * 2
    h0 = 1e-3
    h = np.ascontiguousarray(np.broadcast_to(h0 * np.cos(q * x)[None, :], (16, 32)))
    estar = elastic.e_star(E, NU)
    pbar = 1.2 * estar * q * h0 / 2
    ctx = _ctx(g)
    p, _, info = ctx.contact_solve(torch.from_numpy(h).cuda(), pbar, tol=1e-15, max_iter=500)
    exact = pbar + estar * q * h0 / 2 * np.cos(q * x)[None, :]
    assert np.max(np.abs(p.cpu().numpy() - exact)) < 1e-13 * pbar


def test_flat_surface_elastoplastic_closed_form():
    """Whole chain (contact, DF-SANE, return map, k = 0, Algorithm 1) on a
    flat surface under uniform pressure: uniaxial strain closed form."""
    from paper_1811_11558_amd import EPOptions
    g = grid_dict(8, 8, 4, lz=0.2)
    ctx = _ctx(g)
    st = ctx.new_state()
    pbar = 0.02
    infos = ctx.elastoplastic_solve(torch.zeros((8, 8), dtype=torch.float64, device="cuda"),
                                    [pbar / 3, 2 * pbar / 3, pbar], st,
                                    EPOptions(tol_outer=1e-12, tol_plastic=1e-13, tol_contact=1e-14))
    torch.cuda.synchronize()
    A = np.array([[LAM + 2 * MU, -2 * MU], [2 * MU, -(3 * MU + EH)]])
    e, a = np.linalg.solve(A, [pbar, SY])
    sig = st["sigma"].cpu().numpy()
    epsp = st["eps_p"].cpu().numpy()
    assert np.max(np.abs(sig[2] + pbar)) < 1e-14
    assert np.max(np.abs(epsp[2] + a)) < 1e-12 * a
    assert np.max(np.abs(st["ep"].cpu().numpy() - a)) < 1e-12 * a
    _say(infos)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hertz_ep_16x16x8.npz")


@pytest.mark.parametrize("solver,kdim", [(0, 0), (1, 0), (2, 0), (2, 3), (2, 30)])
def test_hertz_elastoplastic_matches_stored_oracle(solver, kdim):
    """Paraboloid R = 2 L on 16 x 16 x 8 (lz = 0.25 L), two load steps with
    Hertz peak pressures of about 2 and 3 times first yield: the GPU
    Algorithm 1 (DF-SANE, Picard or Newton-Krylov inside; the last also with
    a Krylov space of 3, which truncates most linear solves, and with the
    largest one, 30) reproduces the
    oracle's converged state stored by tests/golden/make_golden.py (computed
    with DF-SANE: the root, not the iteration, is compared)."""
    from paper_1811_11558_amd import EPOptions
    ref = np.load(GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = _ctx(g)
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13,
                                              tol_contact=1e-15, solver=solver, max_plastic=20000,
                                              krylov_dim=kdim))
    torch.cuda.synchronize()
    _say(infos)
    if solver == 2 and kdim == 0:
        # Newton: a handful of steps per plasticity solve, not tens
        for i in infos:
            assert i["plastic_iters"] <= 12 * i["outer_iters"], i
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-11, (k, err)


def test_anderson_outer_reaches_the_stored_fixed_point():
    """Anderson acceleration (depth 5, damping 0.3) of Algorithm 1's outer
    fixed point reaches the state of the oracle's relaxed iteration (stored
    by tests/golden/make_golden.py, outer error below 1e-11), within what the
    two outer tolerances allow, in fewer outer passes (the oracle took 51 and
    57)."""
    import ast
    from paper_1811_11558_amd import EPOptions
    ref = np.load(GOLDEN)
    meta = ast.literal_eval(str(ref["meta"][0]))
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = _ctx(g)
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-12, relax=0.3, tol_plastic=1e-13,
                                              tol_contact=1e-15, max_plastic=20000, anderson_m=5))
    torch.cuda.synchronize()
    passes = [i["outer_iters"] for i in infos]
    _say("outer passes anderson / oracle relaxed", passes, meta["outer"])
    assert all(a < b for a, b in zip(passes, meta["outer"]))
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-8, (k, err)


ROUGH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rough_ep_16x16x8.npz")


@pytest.mark.parametrize("precision,accel,solver", [("fp64", False, 0), ("fp32_refined", True, 0),
                                                   ("fp64", False, 2), ("fp32_refined", True, 2)])
def test_rough_surface_experiment_setting_matches_stored_oracle(precision, accel, solver):
    """The rough-surface experiment's geometry and material (lz = 0.4 L,
    sigma_y = 0.1 E, E_h = 0.01 E, H = 0.8, PSD plateau for 1 <= |k| < 2) on a
    16 x 16 x 8 grid, stored by tests/golden/make_golden.py: the GPU's
    elastic contact pressure under the final load and its Algorithm 1 state
    reproduce the oracle's, and so do both contact areas.  In float64 with
    the oracle's relaxation the bound is rounding (1e-11); with FP32 kernels
    and the accelerated outer/inner iteration it is what the tolerances
    allow (1e-8).  Solver 2 (Newton-Krylov) replaces DF-SANE inside; its
    Jacobian products are float32 in the FP32_REFINED mode."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(ROUGH)
    g = grid_dict(16, 16, 8, lz=0.4)
    ctx = Context(g, 1.0, 0.3, 0.1, 0.01, precision=precision)
    h = torch.from_numpy(ref["h"]).cuda()
    W = list(ref["W"])
    p_el, _, _ = ctx.contact_solve(h, W[-1], tol=1e-15, max_iter=20000)
    torch.cuda.synchronize()
    p_el = p_el.cpu().numpy()
    err = _rel(p_el, ref["p_elastic"])
    _say(precision, "elastic pressure", err)
    assert err < 1e-11
    st = ctx.new_state()
    opts = (EPOptions(tol_outer=1e-12, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15, max_plastic=20000,
                      anderson_m=5, warm_start=1, inner_rel=0.1, solver=solver) if accel else
            EPOptions(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15, max_plastic=20000,
                      solver=solver))
    infos = ctx.elastoplastic_solve(h, W, st, opts)
    torch.cuda.synchronize()
    _say(precision, [(i["outer_iters"], i["r_evals"]) for i in infos])
    bound = 1e-8 if accel else 1e-11
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < bound, (k, err)
    a_el, a_ep = int((p_el > 0).sum()), int((st["traction"][2].cpu().numpy() > 0).sum())
    _say("contact points elastic / elastoplastic", a_el, a_ep)
    assert a_el == int((ref["p_elastic"] > 0).sum())
    assert a_ep == int((ref["traction"][2] > 0).sum())
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_warm_inexact_inner_solves_reach_the_stored_fixed_point(precision):
    """Plasticity solves warm-started from the previous outer pass and solved
    only to 0.1 x the outer error until the outer error is below tol_outer
    (then once more to tol_plastic) end on the state of the oracle's relaxed
    iteration within what the tolerances allow, with fewer residual
    evaluations than full solves from the elastic trial."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    evals = {}
    for warm, rel in ((0, 0.0), (1, 0.1)):
        ctx = Context(g, E, NU, SY, EH, precision=precision)
        st = ctx.new_state()
        infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                        EPOptions(tol_outer=1e-12, relax=0.3, tol_plastic=1e-13,
                                                  tol_contact=1e-15, max_plastic=20000, anderson_m=5,
                                                  warm_start=warm, inner_rel=rel))
        torch.cuda.synchronize()
        evals[warm] = sum(i["r_evals"] for i in infos)
        _say(precision, "warm", warm, "inner_rel", rel, [(i["outer_iters"], i["r_evals"]) for i in infos])
        for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
            err = _rel(st[k].cpu().numpy(), ref[k])
            _say(k, err)
            assert err < 1e-8, (k, err)
        ctx.close()
    assert evals[1] < evals[0], evals


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_residual_graphs_equal_eager(precision):
    """Algorithm 1 on the stored Hertz case with the plasticity residual
    evaluations replayed from captured HIP graphs gives bitwise the same state
    and the same iteration and evaluation counts as launching every kernel
    one by one."""
    from paper_1811_11558_amd import Context, EPOptions
    ref = np.load(GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    out = {}
    for graphs in (1, 0):
        ctx = Context(g, E, NU, SY, EH, precision=precision)
        ctx.set_option(ctx.OPT_GRAPHS, graphs)
        st = ctx.new_state()
        infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                        EPOptions(tol_outer=1e-10, relax=0.3, tol_plastic=1e-12,
                                                  tol_contact=1e-14, max_plastic=20000, anderson_m=5))
        torch.cuda.synchronize()
        out[graphs] = ({k: st[k].cpu().numpy() for k in ("eps_p", "ep", "sigma", "traction", "u3p")},
                       [(i["outer_iters"], i["r_evals"]) for i in infos])
        ctx.close()
    _say(precision, "counts graphs / eager", out[1][1], out[0][1])
    assert out[1][1] == out[0][1]
    for k in out[1][0]:
        assert np.array_equal(out[1][0][k], out[0][0][k]), k


def test_contact_graph_replay_equals_eager():
    """The contact iteration replayed as a captured HIP graph gives bitwise the
    same pressure as launching its kernels one by one (many replays, with
    host reads of the convergence scalar between them)."""
    g = grid_dict(64, 64, 2)
    h = torch.from_numpy(rough_surface(64, 64, hurst=0.8, k_roll=2, k_cut=16, rms_slope=0.1, seed=7)).cuda()
    out = {}
    for graphs in (1, 0, 1):
        ctx = _ctx(g)
        ctx.set_option(3, graphs)
        p, _, info = ctx.contact_solve(h, 0.01, tol=1e-15, max_iter=5000)
        torch.cuda.synchronize()
        out.setdefault(graphs, []).append((p.cpu().numpy(), info["iters"]))
        ctx.close()
    (pg, ig), (pg2, ig2) = out[1]
    (pe, ie), = out[0]
    _say("iterations graph / eager", ig, ie)
    assert ig == ie == ig2
    assert np.array_equal(pg, pe) and np.array_equal(pg, pg2)


def test_newton_krylov_options_are_checked():
    """An unknown solver id or a Krylov dimension beyond 30 is rejected
    before any work; the state is left as it was."""
    from paper_1811_11558_amd import EPOptions
    ref = np.load(GOLDEN)
    g = grid_dict(16, 16, 8, lz=0.25)
    ctx = _ctx(g)
    st = ctx.new_state()
    for bad in (EPOptions(solver=3), EPOptions(solver=2, krylov_dim=31), EPOptions(solver=2, krylov_dim=-1)):
        with pytest.raises(RuntimeError, match="bad options"):
            ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), [float(ref["W"][0])], st, bad)
    assert float(st["ep"].abs().max()) == 0.0
    ctx.close()


def test_elastoplastic_reports_committed_steps_on_failure():
    """elastoplastic_solve commits each converged load step before the next:
    when step 2 cannot converge within max_outer, the call fails with
    FVIM_ENOCONV, info says step 1 was committed and step 2 was not, and the
    state equals that of step 1 solved alone."""
    from paper_1811_11558_amd import EPOptions, FvimError
    from paper_1811_11558_amd import binding as b
    from synth import paraboloid
    g = grid_dict(16, 16, 8, lz=0.25)
    h = torch.from_numpy(paraboloid(g, R=0.5)).cuda()
    opts = EPOptions(tol_outer=1e-10, relax=0.3, tol_plastic=1e-12, tol_contact=1e-14, max_outer=6)
    ctx = _ctx(g)
    ref = ctx.new_state()
    ok = ctx.elastoplastic_solve(h, [1e-6], ref, opts)
    assert ok[0]["committed"] == 1 and ok[0]["outer_iters"] <= 6
    st = ctx.new_state()
    with pytest.raises(FvimError) as ei:
        ctx.elastoplastic_solve(h, [1e-6, 0.002], st, opts)
    assert ei.value.code == b.FVIM_ENOCONV
    infos = ei.value.infos
    assert [i["committed"] for i in infos] == [1, 0]
    assert infos[1]["outer_iters"] == 6
    torch.cuda.synchronize()
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        assert torch.equal(st[k], ref[k]), k
    assert ok[0]["kkt"] >= 0.0 and ok[0]["kkt"] < 1e-10
    ctx.close()


C1 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_32x32x16.npz")


@pytest.mark.parametrize("solver", [0, 2])
def test_c1_paraboloid_matches_stored_oracle(solver):
    """The plain FP64 elastoplastic configuration: 32 x 32 x 16 (lz = 0.25 L),
    paraboloid R = 0.5 L, E = 1, nu = 0.3, sigma_y0 = 0.01, E_h = 0.1, total
    load 0.02 E L^2 in 10 equal cumulative increments, lambda = 0.3, k = 0
    traction included (far beyond first yield: Hertz peak pressure 26
    sigma_y0 at the full load).  The oracle's state after the increments it
    has stored (tests/golden/make_golden.py writes the file after every
    increment) is reproduced by Algorithm 1 with DF-SANE and with
    Newton-Krylov inside, to 1e-11.  The contact solves stop at 1e-14
    (the change of the pressure, relative to the load): at the oracle's
    1e-15 the pressure iteration reaches its rounding floor first on some
    passes of the Newton-Krylov path."""
    from paper_1811_11558_amd import EPOptions
    if not os.path.exists(C1):
        pytest.skip("stored case not written")
    ref = np.load(C1)
    steps = int(ref["steps_done"])
    g = grid_dict(32, 32, 16, lz=0.25)
    ctx = _ctx(g)
    st = ctx.new_state()
    _say("c1: %d increments, solver %d" % (steps, solver))
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"][:steps]), st,
                                    EPOptions(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13, tol_contact=1e-14,
                                              max_outer=400, max_plastic=20000, solver=solver))
    torch.cuda.synchronize()
    _say([(i["outer_iters"], i["r_evals"]) for i in infos])
    assert all(i["committed"] == 1 for i in infos)
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < 1e-11, (k, err)
    ctx.close()


@pytest.mark.parametrize("name,bound", [("hertz_ep_16x16x8", 1e-11), ("hertz_graded_ep_16x16x8", 1e-11),
                                        ("hertz_friction_ep_16x16x8", 1e-11), ("hertz_cerruti_ep_16x16x8", 1e-11),
                                        ("rough_ep_16x16x8", 1e-10)])
def test_newton_coupling_reaches_the_stored_fixed_point(name, bound):
    """The outer Newton-Krylov coupling (coupling = 1) ends on the fixed point
    of Algorithm 1 stored by tests/golden/make_golden.py (the oracle's
    relaxed alternation stopped at |dU3p - dU3p_prev| / |H0| < 1e-11), in far
    fewer passes.  The rough case's stored state lies 2.8e-11 from the
    fixed point (the oracle's own Newton coupling finds that distance), so
    its bound is 1e-10."""
    import ast
    from paper_1811_11558_amd import Context, EPOptions
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gold)
    from make_golden import CASES
    c = CASES[name]
    ref = np.load(os.path.join(gold, name + ".npz"))
    meta = ast.literal_eval(str(ref["meta"][0]))
    nx, ny, nz, lz = c["grid"]
    g = grid_dict(nx, ny, nz, lz=lz)
    m = c["mat"]
    ctx = Context(g, m["E"], m["nu"], m["sigma_y0"], m["E_h"])
    if "z" in ref:
        ctx.set_depth_nodes(ref["z"])
    fr = (dict(mu_f=c["friction"]["mu_f"], q_ratio=c["friction"]["q_ratio"],
               cerruti=int(c["friction"].get("cerruti", False))) if "friction" in c else {})
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-13, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15,
                                              max_plastic=20000, coupling=1, **fr))
    torch.cuda.synchronize()
    _say(name, "newton steps", [i["outer_iters"] for i in infos], "oracle passes", meta["outer"],
         "kkt", [i["kkt"] for i in infos])
    for i, passes in zip(infos, meta["outer"]):
        assert i["outer_err"] < 1e-13 and i["outer_iters"] < passes
        assert i["kkt"] < 1e-10
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < bound, (k, err)
    ctx.close()


def _stored_case(name):
    import ast
    from paper_1811_11558_amd import Context
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gold)
    from make_golden import CASES
    c = CASES[name]
    ref = np.load(os.path.join(gold, name + ".npz"))
    meta = ast.literal_eval(str(ref["meta"][0]))
    nx, ny, nz, lz = c["grid"]
    m = c["mat"]
    ctx = Context(grid_dict(nx, ny, nz, lz=lz), m["E"], m["nu"], m["sigma_y0"], m["E_h"])
    fr = (dict(mu_f=c["friction"]["mu_f"], q_ratio=c["friction"]["q_ratio"]) if "friction" in c else {})
    return ctx, ref, meta, fr


@pytest.mark.parametrize("name,bound", [("hertz_ep_16x16x8", 1e-11), ("hertz_friction_ep_16x16x8", 1e-11),
                                        ("rough_ep_16x16x8", 1e-10)])
def test_switched_coupling_reaches_the_stored_fixed_point(name, bound):
    """coupling = 2 with a slow alternation (relaxation 0.05: hundreds of
    passes to go at pass 20) hands over to the outer Newton-Krylov coupling
    at pass 20, from the alternation's next iterate, and ends on the stored
    fixed point."""
    from paper_1811_11558_amd import EPOptions
    ctx, ref, meta, fr = _stored_case(name)
    st = ctx.new_state()
    infos = ctx.elastoplastic_solve(torch.from_numpy(ref["h"]).cuda(), list(ref["W"]), st,
                                    EPOptions(tol_outer=1e-13, relax=0.05, tol_plastic=1e-13, tol_contact=1e-15,
                                              max_plastic=20000, coupling=2, **fr))
    torch.cuda.synchronize()
    _say(name, "passes + newton steps", [i["outer_iters"] for i in infos], "oracle passes", meta["outer"])
    for i in infos:
        assert i["outer_err"] < 1e-13 and 20 < i["outer_iters"] <= 30
    for k in ("eps_p", "ep", "sigma", "traction", "u3p"):
        err = _rel(st[k].cpu().numpy(), ref[k])
        _say(k, err)
        assert err < bound, (k, err)
    ctx.close()


def test_switched_coupling_without_switch_is_algorithm_1():
    """With the stored cases' relaxation (0.3) the alternation converges at
    a rate that leaves fewer than 100 passes to go, coupling = 2 never hands
    over, and the solve is Algorithm 1's, bit for bit."""
    from paper_1811_11558_amd import EPOptions
    ctx, ref, meta, fr = _stored_case("hertz_friction_ep_16x16x8")
    h = torch.from_numpy(ref["h"]).cuda()
    out = []
    for coupling in (0, 2):
        st = ctx.new_state()
        infos = ctx.elastoplastic_solve(h, list(ref["W"]), st,
                                        EPOptions(tol_outer=1e-13, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15,
                                                  max_plastic=20000, coupling=coupling, **fr))
        torch.cuda.synchronize()
        out.append(([i["outer_iters"] for i in infos], {k: st[k].cpu().numpy() for k in ("eps_p", "traction", "u3p")}))
    _say(out[0][0], out[1][0])
    assert out[0][0] == out[1][0]
    for k in out[0][1]:
        assert np.array_equal(out[0][1][k], out[1][1][k]), k
    ctx.close()


def test_newton_coupling_options_are_checked():
    from paper_1811_11558_amd import EPOptions, FvimError
    g = grid_dict(8, 8, 4, lz=0.2)
    ctx = _ctx(g)
    st = ctx.new_state()
    h = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    for bad in (dict(coupling=3), dict(coupling=1, coupling_krylov=31), dict(coupling=-1)):
        with pytest.raises(FvimError):
            ctx.elastoplastic_solve(h, [0.01], st, EPOptions(**bad))
    # the flat surface: converged at the first pass, no Newton step
    infos = ctx.elastoplastic_solve(h, [0.01, 0.02], st, EPOptions(tol_outer=1e-12, coupling=1))
    assert [i["outer_iters"] for i in infos] == [0, 0]
    ctx.close()

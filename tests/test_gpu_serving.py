"""Continuous-batching server on the GPU: results are the same alone and in a
mix of concurrent requests (bitwise, since every request runs the same
deterministic kernels in its own context), requests overlap on the device,
and admission keeps the device footprint within the budget."""
import sys

import numpy as np
import pytest
import torch

from synth import grid_dict, paraboloid, rough_surface

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _requests():
    out = []
    for i, (n, nz, prec) in enumerate([(32, 16, "fp64"), (64, 32, "fp64"), (32, 8, "fp32_refined"),
                                        (64, 16, "fp32_refined"), (32, 16, "fp64"), (128, 32, "fp64")]):
        g = grid_dict(n, n, nz, lz=0.25)
        if i % 2 == 0:
            h = paraboloid(g, R=2.0)
            W = [0.0005 * (1 + i % 3), 0.001 * (1 + i % 3)]
        else:
            h = rough_surface(n, n, hurst=0.7, k_roll=2, k_cut=n // 4, rms_slope=0.05, seed=i)
            W = [0.002]
        out.append((g, h, W, prec))
    return out


def _opts(accelerated=False, solver=0, mu_f=0.0):
    from paper_1811_11558_amd import EPOptions
    fr = dict(mu_f=mu_f, q_ratio=(0.4, 0.1)) if mu_f > 0 else {}
    if accelerated:     # the serving benchmark's options
        return EPOptions(tol_outer=1e-9, relax=0.3, tol_plastic=1e-11, tol_contact=1e-14, anderson_m=5,
                         warm_start=1, inner_rel=0.1, solver=solver, **fr)
    return EPOptions(tol_outer=1e-9, relax=0.3, tol_plastic=1e-11, tol_contact=1e-14, solver=solver, **fr)


def _run(server, reqs, opts=None):
    opts = opts or _opts()
    ids = [server.submit(g, h, W, precision=prec, opts=opts) for (g, h, W, prec) in reqs]
    return [server.wait(i, (g["ny"], g["nx"])) for i, (g, _, _, _) in zip(ids, reqs)]


@pytest.mark.parametrize("accelerated,solver,mu_f", [(False, 0, 0.0), (True, 0, 0.0), (True, 2, 0.0),
                                                     (True, 0, 0.3)])
def test_results_identical_alone_and_in_mix(accelerated, solver, mu_f):
    """With Algorithm 1's relaxation and with the accelerated options
    (Anderson, warm-started and inexact inner solves, as the serving
    benchmark runs them), the latter also with Newton-Krylov plasticity
    solves (whose host decisions and Krylov workspace are per request) and
    with Coulomb friction in the contact step (per-request tangential
    workspace)."""
    assert torch.cuda.is_available()
    from paper_1811_11558_amd import Server
    reqs = _requests()
    opts = _opts(accelerated, solver, mu_f)
    srv = Server(hbm_budget_bytes=8 << 30, max_slots=4)
    mixed = _run(srv, reqs, opts)
    st = srv.stats()
    srv.close()
    for r in mixed:
        assert r["status"] == 0, r
    # overlap: some request was admitted before an earlier-admitted one finished
    spans = sorted((r["t_admit"], r["t_done"]) for r in mixed)
    overlap = any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))
    _say("spans", spans, "stats", st)
    assert overlap
    for k, req in enumerate(reqs):
        alone = Server(hbm_budget_bytes=8 << 30, max_slots=1)
        a = _run(alone, [req], opts)[0]
        alone.close()
        assert np.array_equal(a["p"], mixed[k]["p"]), k
        assert np.array_equal(a["u3p"], mixed[k]["u3p"]), k
        _say("request", k, "identical alone / in mix; contact fraction", a["contact_fraction"])


def test_admission_respects_budget():
    from paper_1811_11558_amd import Server, request_bytes, FvimError
    g = grid_dict(64, 64, 32, lz=0.25)
    one = request_bytes(g)
    srv = Server(hbm_budget_bytes=int(1.5 * one), max_slots=4)       # room for one at a time
    h = paraboloid(g, R=2.0)
    reqs = [(g, h, [0.0005], "fp64")] * 3
    res = _run(srv, reqs)
    st = srv.stats()
    assert all(r["status"] == 0 for r in res)
    assert st["peak_bytes"] <= st["budget"]
    spans = sorted((r["t_admit"], r["t_done"]) for r in res)
    assert all(spans[k + 1][0] >= spans[k][1] for k in range(len(spans) - 1))   # serialised by memory
    big = grid_dict(512, 512, 96, lz=0.25)
    with pytest.raises(FvimError):
        srv.submit(big, np.zeros((512, 512)), [0.001])
    srv.close()


def test_requests_with_depth_nodes_identical_alone_and_in_mix():
    """Requests may carry their own depth nodes (copied at submission): two
    graded-node requests among uniform ones give the same result alone and
    in the mix, and differ from the same request on uniform nodes."""
    from paper_1811_11558_amd import Server
    assert torch.cuda.is_available()
    reqs = _requests()[:4]
    zs = []
    for k, (g, h, W, prec) in enumerate(reqs):
        nz = g["nz"]
        z = None
        if k % 2 == 0:
            z = g["lz"] * (np.arange(nz) / (nz - 1)) ** 2
            z[-1] = g["lz"]
        zs.append(z)
    opts = _opts(True)

    def run(server, items):
        ids = [server.submit(g, h, W, precision=prec, opts=opts, z=z) for (g, h, W, prec), z in items]
        return [server.wait(i, (g["ny"], g["nx"])) for i, ((g, _, _, _), _) in zip(ids, items)]

    srv = Server(hbm_budget_bytes=8 << 30, max_slots=4)
    mixed = run(srv, list(zip(reqs, zs)))
    srv.close()
    for r in mixed:
        assert r["status"] == 0, r
    for k in range(len(reqs)):
        alone = Server(hbm_budget_bytes=8 << 30, max_slots=1)
        a = run(alone, [(reqs[k], zs[k])])[0]
        alone.close()
        assert np.array_equal(a["p"], mixed[k]["p"]), k
        assert np.array_equal(a["u3p"], mixed[k]["u3p"]), k
    uni = Server(hbm_budget_bytes=8 << 30, max_slots=1)
    u0 = run(uni, [(reqs[0], None)])[0]
    uni.close()
    assert not np.array_equal(u0["u3p"], mixed[0]["u3p"])


def test_served_results_match_the_stored_oracle_cases():
    """The stored oracle cases (Hertz, the rough-surface experiment's setting,
    graded depth nodes, Coulomb friction, Cerruti-coupled friction under the
    outer Newton coupling, Goodman friction under the switched coupling
    with a slow relaxation, adhesion; written by tests/golden/make_golden.py
    from the oracle alone) submitted to the server in one mix with rough
    requests of other grids, the Hertz case twice so that a slot reuses its
    context: the served pressure and plastic surface displacement equal the
    oracle's within 1e-11."""
    import os
    from paper_1811_11558_amd import EPOptions, Server
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, gold)
    from make_golden import CASES
    cases = [("hertz_ep_16x16x8", {}), ("rough_ep_16x16x8", {}), ("hertz_graded_ep_16x16x8", {}),
             ("hertz_friction_ep_16x16x8", {}), ("hertz_ep_16x16x8", {}),
             ("hertz_cerruti_ep_16x16x8", dict(coupling=1, tol_outer=1e-13)),
             ("hertz_friction_ep_16x16x8", dict(coupling=2, relax=0.05, tol_outer=1e-13)),
             ("hertz_adhesion_ep_16x16x8", dict(tol_contact=1e-14))]
    srv = Server(hbm_budget_bytes=8 << 30, max_slots=3)
    ids = []
    for i, (name, extra) in enumerate(cases):
        c = CASES[name]
        ref = np.load(os.path.join(gold, name + ".npz"))
        nx, ny, nz, lz = c["grid"]
        g = grid_dict(nx, ny, nz, lz=lz)
        fr = (dict(mu_f=c["friction"]["mu_f"], q_ratio=c["friction"]["q_ratio"],
                   cerruti=int(c["friction"].get("cerruti", False))) if "friction" in c else {})
        if "adhesion" in c:
            fr["adhesion"] = tuple(c["adhesion"])
        kw = dict(tol_outer=1e-11, relax=0.3, tol_plastic=1e-13, tol_contact=1e-15, max_plastic=20000, **fr)
        kw.update(extra)
        opts = EPOptions(**kw)
        m = c["mat"]
        ids.append((name, ref, g, srv.submit(g, ref["h"], list(ref["W"]), E=m["E"], nu=m["nu"],
                                             sigma_y0=m["sigma_y0"], E_h=m["E_h"], opts=opts,
                                             z=ref["z"] if "z" in ref else None)))
        # other traffic between the stored cases
        n = 32 * (1 + i % 2)
        go = grid_dict(n, n, 16, lz=0.25)
        ho = rough_surface(n, n, hurst=0.7, k_roll=2, k_cut=n // 4, rms_slope=0.05, seed=100 + i)
        srv.submit(go, ho, [0.002], opts=_opts(True))
    for name, ref, g, rid in ids:
        r = srv.wait(rid, (g["ny"], g["nx"]))
        assert r["status"] == 0, (name, r)
        ep = np.linalg.norm(r["p"] - ref["traction"][2]) / np.linalg.norm(ref["traction"][2])
        eu = np.linalg.norm(r["u3p"] - ref["u3p"]) / np.linalg.norm(ref["u3p"])
        _say("served", name, "p", ep, "u3p", eu, "outer", r["info"]["outer_iters"])
        assert ep < 1e-11 and eu < 1e-11, (name, ep, eu)
    srv.close()

"""Writes the stored oracle results used by the GPU solver tests.

Calls only ``oracle/`` and ``synth/``.  Run from the repository root:
    python tests/golden/make_golden.py [name ...]
Each case is the FP64 oracle's Algorithm 1 (Sec. 5.2) on a seeded
synthetic input; the GPU solver must reproduce the stored state.
    python tests/golden/make_golden.py --resume c1_32x32x16
continues a checkpointed case from the increments its file already holds
(the state carries over exactly as inside one run).
"""
import ast
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import contact as oc  # noqa: E402
from oracle import coupling as cp  # noqa: E402
from synth import grid_dict, paraboloid, rough_surface  # noqa: E402

CASES = {
    # paraboloid R = 2 L on 16 x 16 x 8 (lz = 0.25 L), E = 1, nu = 0.3,
    # sigma_y0 = 0.01, E_h = 0.1; two cumulative loads with Hertz peak
    # pressures of about 2 and 3 times the first-yield pressure 1.6 sigma_y0
    "hertz_ep_16x16x8": dict(grid=(16, 16, 8, 0.25), R=2.0, W=[0.001, 0.002], relax=0.3,
                             mat=dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1)),
    # the rough-surface experiment's geometry and material (Sec. on rough
    # surface contact and its appendix: lz = 0.4 L, H = 0.8, PSD plateau for
    # 1 <= |k| < 2, sigma_y = 0.1 E, E_h = 0.01 E) on 16 x 16 x 8: cut-off
    # k = 4, rms slope 0.5, seed 3, two cumulative mean pressures up to
    # 0.01 E (mean contact pressure about 2.5 sigma_y); the elastic contact
    # solution under the final load is stored as well
    "rough_ep_16x16x8": dict(grid=(16, 16, 8, 0.4), rough=dict(hurst=0.8, k_roll=2, k_cut=4, rms_slope=0.5, seed=3),
                             W=[0.005, 0.01], relax=0.3, mat=dict(E=1.0, nu=0.3, sigma_y0=0.1, E_h=0.01)),
    # the Hertz case with Coulomb friction in the contact step: mu_f = 0.3,
    # tangential force 0.5 mu_f W along x and 0.2 mu_f W along y at each load
    "hertz_friction_ep_16x16x8": dict(grid=(16, 16, 8, 0.25), R=2.0, W=[0.001, 0.002], relax=0.3,
                                      mat=dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1),
                                      friction=dict(mu_f=0.3, q_ratio=(0.5, 0.2))),
    # the friction case with the normal and tangential contact problems
    # coupled through the Boussinesq-Cerruti cross terms
    "hertz_cerruti_ep_16x16x8": dict(grid=(16, 16, 8, 0.25), R=2.0, W=[0.001, 0.002], relax=0.3,
                                     mat=dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1),
                                     friction=dict(mu_f=0.3, q_ratio=(0.5, 0.2), cerruti=True)),
    # the Hertz case with adhesion in the contact step: Dugdale cohesive
    # zone of stress sigma0 = 0.01 E (the yield stress) and range h0 = 0.003 L
    "hertz_adhesion_ep_16x16x8": dict(grid=(16, 16, 8, 0.25), R=2.0, W=[0.001, 0.002], relax=0.3,
                                      mat=dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1),
                                      adhesion=(0.01, 0.003)),
    # the Hertz case on depth nodes graded toward the surface,
    # z_i = lz (i / (nz - 1))^2
    "hertz_graded_ep_16x16x8": dict(grid=(16, 16, 8, 0.25), R=2.0, W=[0.001, 0.002], relax=0.3,
                                    mat=dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1), graded=2.0),
    # the plain FP64 elastoplastic configuration: 32 x 32 x 16, lz = 0.25 L,
    # paraboloid R = 0.5 L centred on node (16, 16), E = 1, nu = 0.3,
    # sigma_y0 = 0.01, E_h = 0.1, total load W = 0.02 E L^2 in 10 equal
    # cumulative increments, lambda = 0.3, k = 0 traction included.  The file
    # is rewritten after every increment; "steps_done" says how many of the
    # loads the stored state has taken.
    "c1_32x32x16": dict(grid=(32, 32, 16, 0.25), R=0.5, W=[0.002 * (i + 1) for i in range(10)], relax=0.3,
                        mat=dict(E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1), checkpoint=True),
}
# Standard under-relaxation (the printed overwrite of the relaxed update
# oscillates on these cases; see the design notes).
OPTS = dict(tol_outer=1e-11, tol_plastic=1e-13, tol_contact=1e-15, max_outer=400, max_plastic=2000,
            max_contact=20000, literal=False)


def contact_options(c):
    """Friction and adhesion settings of a case, as elastoplastic_solve takes them."""
    out = dict(c.get("friction", {}))
    if "adhesion" in c:
        out["adhesion"] = c["adhesion"]
    return out


def run(name, resume=False):
    c = CASES[name]
    nx, ny, nz, lz = c["grid"]
    g = grid_dict(nx, ny, nz, lz=lz)
    if "graded" in c:
        z = lz * (np.arange(nz) / (nz - 1)) ** c["graded"]
        z[-1] = lz
        g["z"] = z
    mat = c["mat"]
    if "rough" in c:
        h = rough_surface(nx, ny, **c["rough"])
    else:
        h = paraboloid(g, R=c["R"])
    extra = {}
    if "rough" in c:
        p_el, _, _ = oc.contact_solve(h, c["W"][-1], g, mat["E"], mat["nu"], tol=1e-15, max_iter=20000)
        extra["p_elastic"] = p_el
    st = cp.new_state(g)
    if "z" in g:
        extra["z"] = g["z"]
    t0 = time.time()
    if c.get("checkpoint"):
        # one increment at a time (the state carries over, as inside one call)
        infos = []
        first = 0
        path = os.path.join(HERE, name + ".npz")
        if resume and os.path.exists(path):
            d = np.load(path)
            first = int(d["steps_done"])
            for key in st:
                st[key] = np.array(d[key])
            m = ast.literal_eval(str(d["meta"][0]))
            t0 -= m["seconds"]
            infos = [{"outer_iters": o, "outer_err": e, "plastic": pl}
                     for o, e, pl in zip(m["outer"], m["outer_err"], m["plastic"])]
        for k, W in enumerate(c["W"]):
            if k < first:
                continue
            infos += cp.elastoplastic_solve(g, mat, h, [W], st, relax=c["relax"], **OPTS, **contact_options(c))
            save(name, c, g, h, st, infos, time.time() - t0, extra, k + 1)
            print(name, "step %d: %.1f s, %d outer passes" % (k + 1, time.time() - t0, infos[-1]["outer_iters"]),
                  flush=True)
        return
    infos = cp.elastoplastic_solve(g, mat, h, c["W"], st, relax=c["relax"], **OPTS, **contact_options(c))
    save(name, c, g, h, st, infos, time.time() - t0, extra, len(c["W"]))
    print(name, "%.1f s" % (time.time() - t0), [i["outer_iters"] for i in infos])


def save(name, c, g, h, st, infos, dt, extra, steps_done):
    meta = np.array([repr({"case": c, "opts": OPTS, "seconds": dt,
                           "outer": [i["outer_iters"] for i in infos],
                           "outer_err": [i["outer_err"] for i in infos],
                           "plastic": [i["plastic"] for i in infos]})])
    more = dict(extra)
    if c.get("checkpoint"):
        more["steps_done"] = np.array(steps_done)
    path = os.path.join(HERE, name + ".npz")
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, h=h, W=np.array(c["W"]), meta=meta, **{k: v for k, v in st.items()}, **more)
    os.replace(tmp, path)        # readers never see a half-written file


if __name__ == "__main__":
    args = sys.argv[1:]
    resume = "--resume" in args
    args = [a for a in args if a != "--resume"]
    for n in (args or list(CASES)):
        run(n, resume=resume)

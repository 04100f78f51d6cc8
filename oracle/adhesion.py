"""Adhesive normal contact with a rigid surface (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. 5.1 says adhesion, like friction, can be included in the contact step;
the paper gives no model.  This module takes the Dugdale cohesive zone of
Maugis's adhesion theory, written for the discrete periodic surface:

* the surfaces attract with a constant stress sigma0 wherever the gap g is
  at most the range h0, the contact zone (g = 0) included; the work of
  adhesion is w = sigma0 h0;
* where they touch, a repulsive pressure p_c >= 0 acts, with g >= 0 and
  p_c g = 0 (the Hertz-Signorini-Moreau conditions of Sec. 2 on p_c);
* the traction on the body is p = p_c - sigma0 1[g <= h0] (force per area,
  +e3 into the body), and the load is dA sum p = W (eqn total_pressure).

For a given cohesive set C the adhesive traction is known, and the
problem for p_c is the frictionless contact problem of ``contact``: the
displacement of -sigma0 1_C moves the surface towards the rigid one, so
p_c solves contact_solve on the surface h + M[sigma0 1_C] under the load
W + sigma0 dA |C|, and the gap of that solve is the gap of the whole
traction.  The set is found by fixed point: starting from C = {} (the
non-adhesive solution), C <- {g <= h0} until the set repeats, each contact
solve warm-started from the last.  Adhesive contact can have several
solutions (hysteresis); this sequence picks one deterministically.
"""
import numpy as np

from . import contact as oc


def adhesive_contact_solve(grid, E, nu, h, W, sigma0, h0, tol=1e-14, max_iter=200, max_contact=5000):
    """Returns (p, gap, info): the total traction p = p_c - sigma0 1_C
    (ny, nx), the gap (>= 0, 0 where p_c > 0) and info with the set
    iterations, the cohesive set C, the repulsive pressure p_c and the last
    contact record.  Raises if the set has not repeated after max_iter
    solves."""
    nx, ny = grid['nx'], grid['ny']
    dA = grid['lx'] * grid['ly'] / (nx * ny)
    h = np.asarray(h, dtype=float)
    sym = oc.surface_compliance_symbol(grid, E, nu)
    C = np.zeros((ny, nx), dtype=bool)
    pc = None
    for k in range(1, max_iter + 1):
        h2 = h + oc.apply_compliance(sigma0 * C.astype(float), sym)
        W2 = W + sigma0 * dA * np.count_nonzero(C)
        pc, gap, cinfo = oc.contact_solve(h2, W2, grid, E, nu, tol=tol, max_iter=max_contact, p0=pc)
        Cn = gap <= h0
        if np.array_equal(Cn, C):
            break
        C = Cn
    else:
        raise RuntimeError("cohesive set did not settle in %d solves" % max_iter)
    p = pc - sigma0 * C
    info = {"iters": k, "cohesive": C, "p_c": pc, "contact": cinfo,
            "cohesive_fraction": float(np.mean(C)), "contact_fraction": float(np.mean(pc > 0)),
            "adhesive_force": float(sigma0 * dA * np.count_nonzero(C))}
    return p, gap, info

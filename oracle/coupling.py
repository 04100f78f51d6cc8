"""Incremental plasticity fixed point and Algorithm 1 (oracle).

Test infrastructure only (see ``oracle/__init__``).

* ``plasticity``: solves R[d_eps] = 0 with
  R[d_eps] = d_eps - grad_s M[dT] - grad_s N[C : d_eps_p(d_eps; S_n)]
  (eqn incremental_strain), d_eps_p from the radial return, by the DF-SANE
  spectral residual method of Sec. 4.3 or by plain fixed-point (Picard)
  iteration d_eps <- d_eps - R[d_eps].
* ``dfsane``: La Cruz, Martinez and Raydan (2006): direction -sigma_k F,
  sigma_k = <s, s>/<s, y> of the last step s and residual change y, clipped
  to [1e-10, 1e10] in absolute value, sigma_0 = 1; nonmonotone two-sided
  line search accepting x +/- alpha d when
  |F|^2 <= max(last 10 |F|^2) + eta_k - gamma alpha^2 |F_k|^2,
  eta_k = |F_0| / (1 + k)^2, gamma = 1e-4, step reduced by safeguarded
  quadratic interpolation into [0.1, 0.5] of the previous alpha.  The paper
  gives the iteration but none of these constants; these are the published
  defaults.
* ``newton_krylov``: Newton's method on the same R with the consistent
  tangent J v = v - grad_s N[C : d(d_eps_p)/d(d_eps) v] (the alternative
  Sec. 4.3 names): each linear system J delta = -R solved by GMRES (SciPy)
  to a tight relative tolerance, the step halved until |R| decreases by the
  Armijo factor 1 - 1e-4 alpha.
* ``elastoplastic_solve``: Algorithm 1 over cumulative loads.  The printed
  algorithm overwrites the relaxed surface correction with the unrelaxed one
  at the end of each pass (``literal=True``); by default the relaxed value is
  kept (plain under-relaxation), which has the same fixed point and, unlike
  the printed form, converges on the Hertz cases of the tests.
"""
import numpy as np

from . import contact as oc
from . import adhesion as ad
from . import friction as fr
from . import operators as ops
from . import plasticity as pl


def dfsane(F, x0, inner, tol_abs, max_iter=500, memory=10, gamma=1e-4,
           sig_min=1e-10, sig_max=1e10, tau_min=0.1, tau_max=0.5):
    """Root of F by DF-SANE.  inner(a, b) is the scalar product.

    Returns (x, Fx, info).  Stops when |F| <= tol_abs."""
    x = x0
    Fx = F(x)
    nevals = 1
    f = inner(Fx, Fx)
    f0n = np.sqrt(f)
    hist = [f]
    sigma = 1.0
    k = 0
    while np.sqrt(f) > tol_abs and k < max_iter:
        d = -sigma * Fx
        eta = f0n / (1.0 + k) ** 2
        fbar = max(hist[-memory:])
        ap = am = 1.0
        while True:
            xp = x + ap * d
            Fp = F(xp)
            nevals += 1
            fp = inner(Fp, Fp)
            if fp <= fbar + eta - gamma * ap * ap * f:
                xn, Fn, fn = xp, Fp, fp
                break
            xm = x - am * d
            Fm = F(xm)
            nevals += 1
            fm = inner(Fm, Fm)
            if fm <= fbar + eta - gamma * am * am * f:
                xn, Fn, fn = xm, Fm, fm
                break
            at = ap * ap * f / (fp + (2.0 * ap - 1.0) * f)
            ap = min(max(at, tau_min * ap), tau_max * ap)
            at = am * am * f / (fm + (2.0 * am - 1.0) * f)
            am = min(max(at, tau_min * am), tau_max * am)
        s = xn - x
        y = Fn - Fx
        sy = inner(s, y)
        ss = inner(s, s)
        if sy == 0.0:
            sigma = sig_max
        else:
            sigma = ss / sy
            sgn = 1.0 if sigma >= 0 else -1.0
            sigma = sgn * min(max(abs(sigma), sig_min), sig_max)
        x, Fx, f = xn, Fn, fn
        hist.append(f)
        k += 1
    return x, Fx, {"iters": k, "evals": nevals, "res": float(np.sqrt(f))}


def newton_krylov(F, J, x0, inner, tol_abs, max_iter=50, lin_rtol=1e-12):
    """Root of F by Newton's method.  J(x, v) is the derivative of F at x
    applied to v; inner(a, b) the scalar product of the stopping test.

    Returns (x, Fx, info) with the residual norm after every iteration in
    info["history"]."""
    from scipy.sparse.linalg import LinearOperator, gmres
    x = x0
    Fx = F(x)
    f = np.sqrt(inner(Fx, Fx))
    hist = [f]
    nevals, k = 1, 0
    shape = x.shape
    while f > tol_abs and k < max_iter:
        xk = x
        A = LinearOperator((x.size, x.size), dtype=float,
                           matvec=lambda v: J(xk, v.reshape(shape)).ravel())
        d, status = gmres(A, -Fx.ravel(), rtol=lin_rtol, atol=0.0, restart=200, maxiter=20)
        d = d.reshape(shape)
        a = 1.0
        while True:
            xn = x + a * d
            Fn = F(xn)
            nevals += 1
            fn = np.sqrt(inner(Fn, Fn))
            if fn <= (1.0 - 1e-4 * a) * f or a < 1e-10:
                break
            a *= 0.5
        x, Fx, f = xn, Fn, fn
        hist.append(f)
        k += 1
    return x, Fx, {"iters": k, "evals": nevals, "res": float(f), "history": hist}


def plasticity(grid, mat, dT, state, tol=1e-13, max_iter=500, solver="dfsane", k0_policy="include"):
    """Strain increment of one load increment with tractions increment dT.

    mat: dict E, nu, sigma_y0, E_h.  state: dict eps_p, ep, sigma (arrays).
    Returns dict d_eps, d_eps_p, d_ep, sigma, info."""
    E, nu = mat['E'], mat['nu']
    b = ops.boussinesq_apply(grid, E, nu, dT, k0_policy=k0_policy)['strain']

    def rmap(de):
        return pl.return_map(de, state['sigma'], state['ep'], E, nu, mat['sigma_y0'], mat['E_h'])

    def R(de):
        dep, _, _ = rmap(de)
        return de - b - ops.mindlin_apply(grid, E, nu, dep, k0_policy=k0_policy)['strain']

    inner = lambda a, c: pl.inner(a, c, grid)
    tol_abs = tol * max(np.sqrt(inner(b, b)), 1e-300)
    if solver == "dfsane":
        de, Rv, info = dfsane(R, b.copy(), inner, tol_abs, max_iter=max_iter)
    elif solver == "newton":
        def Jv(de, v):
            t = pl.return_map_tangent(de, state['sigma'], state['ep'], E, nu, mat['sigma_y0'], mat['E_h'], v)
            return v - ops.mindlin_apply(grid, E, nu, t, k0_policy=k0_policy)['strain']
        de, Rv, info = newton_krylov(R, Jv, b.copy(), inner, tol_abs, max_iter=max_iter)
    else:
        de = b.copy()
        Rv = R(de)
        it = 0
        while np.sqrt(inner(Rv, Rv)) > tol_abs and it < max_iter:
            de = de - Rv
            Rv = R(de)
            it += 1
        info = {"iters": it, "evals": it + 1, "res": float(np.sqrt(inner(Rv, Rv)))}
    dep, dp, sig = rmap(de)
    return {"d_eps": de, "d_eps_p": dep, "d_ep": dp, "sigma": sig, "info": info}


def new_state(grid):
    nx, ny, nz = grid['nx'], grid['ny'], grid['nz']
    return {"eps_p": np.zeros((6, nz, ny, nx)), "ep": np.zeros((nz, ny, nx)),
            "sigma": np.zeros((6, nz, ny, nx)), "traction": np.zeros((3, ny, nx)),
            "u3p": np.zeros((ny, nx))}


def elastoplastic_solve(grid, mat, h, W_steps, state, tol_outer=1e-12, relax=0.3,
                        tol_plastic=1e-13, tol_contact=1e-14, max_outer=500,
                        max_plastic=500, max_contact=5000, solver="dfsane", literal=False,
                        k0_policy="include", mu_f=0.0, q_ratio=(0.0, 0.0), tol_friction=1e-13, cerruti=False,
                        adhesion=None):
    """Algorithm 1 for each cumulative load in W_steps; state updated in place.

    With mu_f > 0 the contact step also carries Coulomb friction: after the
    normal solve, the partial-slip tangential traction for the total
    tangential force Q = q_ratio mu_f W (``friction.tangential_solve``,
    normal and tangential problems uncoupled) joins the traction T, so the
    plasticity sees it through the Boussinesq-Cerruti operator.  The
    tangential problem is solved in total form at each load, which is the
    Cattaneo-Mindlin reading for monotonic proportional loading.  With
    cerruti=True the normal and tangential solves are coupled through the
    Boussinesq-Cerruti cross terms (``friction.frictional_contact_solve``,
    warm-started from the previous pass's traction within a step).
    With adhesion = (sigma0, h0) the contact step is the adhesive contact of
    ``adhesion.adhesive_contact_solve`` (Dugdale cohesive zone, solved
    afresh at each pass) and T3 is its total traction (negative in the
    cohesive zone); not combined with friction.

    Returns a list of per-step info dicts."""
    E, nu = mat['E'], mat['nu']
    infos = []
    for W in W_steps:
        H0 = h - state['u3p']
        hnorm = np.linalg.norm(H0)
        if hnorm == 0.0:
            hnorm = 1.0
        T_n = state['traction']
        dU_prev = np.zeros_like(H0)
        H = H0
        p = None
        res = None
        err = np.inf
        k = 0
        hist = []
        q_prev = None
        for k in range(1, max_outer + 1):
            T = np.zeros_like(T_n)
            if adhesion is not None:
                if mu_f > 0.0:
                    raise ValueError("adhesion with friction is not supported")
                p, _, ainfo = ad.adhesive_contact_solve(grid, E, nu, H, W, adhesion[0], adhesion[1], tol=tol_contact,
                                                        max_contact=max_contact)
                cinfo = ainfo["contact"]
                T[2] = p
            elif mu_f > 0.0 and cerruti:
                Q = np.asarray(q_ratio, dtype=float) * mu_f * W
                p, T[:2], finfo = fr.frictional_contact_solve(
                    grid, E, nu, H, W, Q, mu_f, coupled=True, tol=tol_friction, tol_contact=tol_contact,
                    tol_friction=tol_friction, max_contact=max_contact, p0=p, q0=q_prev)
                cinfo = finfo["contact"]
                q_prev = T[:2].copy()
                T[2] = p
            else:
                p, _, cinfo = oc.contact_solve(H, W, grid, E, nu, tol=tol_contact, max_iter=max_contact, p0=p)
                T[2] = p
            if mu_f > 0.0 and not cerruti:
                Q = np.asarray(q_ratio, dtype=float) * mu_f * W
                T[:2], _ = fr.tangential_solve(grid, E, nu, p, Q, mu_f, tol=tol_friction)
            res = plasticity(grid, mat, T - T_n, state, tol=tol_plastic, max_iter=max_plastic,
                             solver=solver, k0_policy=k0_policy)
            dU = ops.mindlin_apply(grid, E, nu, res['d_eps_p'], k0_policy=k0_policy)['surf_u3']
            err = np.linalg.norm(dU - dU_prev) / hnorm
            hist.append(float(err))
            relaxed = dU_prev + relax * (dU - dU_prev)
            H = H0 - relaxed
            dU_prev = dU if literal else relaxed
            if err < tol_outer:
                break
        state['eps_p'] = state['eps_p'] + res['d_eps_p']
        state['ep'] = state['ep'] + res['d_ep']
        state['sigma'] = res['sigma']
        state['traction'] = T
        state['u3p'] = state['u3p'] + dU
        infos.append({"outer_iters": k, "outer_err": float(err), "plastic": res['info'],
                      "contact": cinfo, "p": p, "history": hist})
    return infos


def outer_map(grid, mat, H0, W, state, x, p0=None, tol_plastic=1e-13, tol_contact=1e-14, max_plastic=500,
              max_contact=5000, solver="dfsane", k0_policy="include", mu_f=0.0, q_ratio=(0.0, 0.0),
              tol_friction=1e-13, cerruti=False, q0=None, adhesion=None):
    """One pass of Algorithm 1 as a map of the surface correction x: the
    contact step on the modified surface H0 - x (warm-started from p0),
    with friction the tangential step, the plasticity step for the traction
    increment, and the surface displacement of N[C : d_eps_p] it produces.
    Returns (G(x), aux) with aux the pass's pressure, traction, plasticity
    result and contact record.  With cerruti=True and friction the contact
    step is the coupled normal-tangential solve, warm-started from (p0, q0)."""
    E, nu = mat['E'], mat['nu']
    T = np.zeros_like(state['traction'])
    if adhesion is not None:
        if mu_f > 0.0:
            raise ValueError("adhesion with friction is not supported")
        p, _, ainfo = ad.adhesive_contact_solve(grid, E, nu, H0 - x, W, adhesion[0], adhesion[1], tol=tol_contact,
                                                max_contact=max_contact)
        cinfo = ainfo["contact"]
        T[2] = p
    elif mu_f > 0.0 and cerruti:
        Q = np.asarray(q_ratio, dtype=float) * mu_f * W
        p, T[:2], finfo = fr.frictional_contact_solve(
            grid, E, nu, H0 - x, W, Q, mu_f, coupled=True, tol=tol_friction, tol_contact=tol_contact,
            tol_friction=tol_friction, max_contact=max_contact, p0=p0, q0=q0)
        cinfo = finfo["contact"]
        T[2] = p
    else:
        p, _, cinfo = oc.contact_solve(H0 - x, W, grid, E, nu, tol=tol_contact, max_iter=max_contact, p0=p0)
        T[2] = p
    if mu_f > 0.0 and not cerruti:
        Q = np.asarray(q_ratio, dtype=float) * mu_f * W
        T[:2], _ = fr.tangential_solve(grid, E, nu, p, Q, mu_f, tol=tol_friction)
    res = plasticity(grid, mat, T - state['traction'], state, tol=tol_plastic, max_iter=max_plastic,
                     solver=solver, k0_policy=k0_policy)
    dU = ops.mindlin_apply(grid, E, nu, res['d_eps_p'], k0_policy=k0_policy)['surf_u3']
    return dU, {"p": p, "T": T, "res": res, "contact": cinfo}


def elastoplastic_solve_newton(grid, mat, h, W_steps, state, tol_outer=1e-12, fd_rel=1e-7, krylov=20,
                               max_newton=50, tol_plastic=1e-13, tol_contact=1e-14, max_plastic=500,
                               max_contact=5000, solver="dfsane", k0_policy="include", mu_f=0.0,
                               q_ratio=(0.0, 0.0), tol_friction=1e-13, cerruti=False, adhesion=None):
    """The fixed point of Algorithm 1 by Newton's method instead of relaxed
    alternation: for each cumulative load, F(x) = G(x) - x = 0 with G the
    pass map ``outer_map`` of the surface correction x, each Newton system
    (J_G - I) d = -F solved by GMRES (SciPy) with the products J_G v formed
    by a forward difference (G(x + h v) - G(x)) / h, h = fd_rel (1 + |x|)
    / |v| (Jacobian-free Newton-Krylov, Knoll and Keyes 2004), and the step
    halved until |F| decreases by the Armijo factor 1 - 1e-4 alpha.  The
    stopping test is Algorithm 1's: |G(x) - x| / |H0| < tol_outer.  The
    state is committed from the pass at the final x, as in Algorithm 1.
    Returns per-step records (newton steps, pass-map evaluations, error)."""
    from scipy.sparse.linalg import LinearOperator, gmres
    kw = dict(tol_plastic=tol_plastic, tol_contact=tol_contact, max_plastic=max_plastic,
              max_contact=max_contact, solver=solver, k0_policy=k0_policy, mu_f=mu_f, q_ratio=q_ratio,
              tol_friction=tol_friction, cerruti=cerruti, adhesion=adhesion)
    infos = []
    for W in W_steps:
        H0 = h - state['u3p']
        hnorm = np.linalg.norm(H0)
        if hnorm == 0.0:
            hnorm = 1.0
        shape = H0.shape
        x = np.zeros_like(H0)
        Gx, aux = outer_map(grid, mat, H0, W, state, x, **kw)
        nevals = 1
        F = Gx - x
        fn = np.linalg.norm(F)
        k = 0
        while fn / hnorm >= tol_outer and k < max_newton:
            xb, Gb, pb, qb = x, Gx, aux["p"], aux["T"][:2].copy()

            def jv(v, xb=xb, Gb=Gb, pb=pb, qb=qb):
                nonlocal nevals
                v = v.reshape(shape)
                nv = np.linalg.norm(v)
                if nv == 0.0:
                    return np.zeros(v.size)
                hs = fd_rel * (1.0 + np.linalg.norm(xb)) / nv
                Gv, _ = outer_map(grid, mat, H0, W, state, xb + hs * v, p0=pb, q0=qb if cerruti else None, **kw)
                nevals += 1
                return ((Gv - Gb) / hs - v).ravel()

            A = LinearOperator((x.size, x.size), dtype=float, matvec=jv)
            d, _ = gmres(A, -F.ravel(), rtol=1e-3, atol=0.0, restart=krylov, maxiter=1)
            d = d.reshape(shape)
            a = 1.0
            while True:
                xn = xb + a * d
                Gn, auxn = outer_map(grid, mat, H0, W, state, xn, p0=pb, q0=qb if cerruti else None, **kw)
                nevals += 1
                Fn = Gn - xn
                if np.linalg.norm(Fn) <= (1.0 - 1e-4 * a) * fn or a < 1e-4:
                    break
                a *= 0.5
            x, Gx, aux, F, fn = xn, Gn, auxn, Fn, np.linalg.norm(Fn)
            k += 1
        res = aux["res"]
        state['eps_p'] = state['eps_p'] + res['d_eps_p']
        state['ep'] = state['ep'] + res['d_ep']
        state['sigma'] = res['sigma']
        state['traction'] = aux["T"]
        state['u3p'] = state['u3p'] + Gx
        infos.append({"newton": k, "evals": nevals, "outer_err": float(fn / hnorm), "p": aux["p"],
                      "contact": aux["contact"]})
    return infos

"""Tangential (frictional) contact under a given normal pressure (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. 5.1 notes that friction can be added to the contact step.  The paper
gives no formulation; this module takes the classical one:

* Coulomb's law with friction coefficient mu_f: the tangential traction q
  (2 components, the tangential part of the applied surface traction of the
  operators) satisfies |q| <= mu_f p at every surface point.
* Normal and tangential problems are uncoupled (Goodman's approximation):
  the normal pressure p is given (from the frictionless solve), and the
  tangential surface displacement is u_t = C[q] with C the tangential block
  of the half-space surface compliance.  Per in-plane mode k, with
  n = k / |k|, C = (2 (1 + nu) / (E |k|)) (I - nu n n^T) (the Cerruti
  surface displacement).  The k = 0 mode is dropped as in the normal
  problem (the mean displacement is the free rigid shift).  On a Nyquist
  line the coupling term is the average over the sign replicas, which
  removes n1 n2 there (the reading of the operators).
* Load control: the total tangential force is Q, dA sum q = Q.

The traction is the minimiser of the complementary energy
    1/2 <q, C q>  over  |q_i| <= mu_f p_i,  dA sum q_i = Q,
whose optimality conditions are the stick/slip conditions: u_t = delta
(one rigid shift) where |q| < mu_f p, and u_t - delta = -s q / |q|, s >= 0,
where the traction is on the friction limit.

Coupled form (``frictional_contact_solve`` with coupled=True): for nu < 1/2
the Boussinesq-Cerruti surface response also has cross terms, per mode
u_a = K_a(k) t3 (tangential displacement from the pressure) and
u3 = conj(K_a(k)) t_a (normal displacement from the tangential traction),
K_a = i (1 - 2 nu) n_a / (2 mu |k|), zero at k = 0 and on the Nyquist line
of axis a (odd in k_a).  The normal problem then sees the surface
h - u3[q] and the tangential problem the extra displacement u_t[p]; the
pair (p, q) is found by alternating the two solves (each warm-started from
the previous one) until neither changes.

``tangential_solve`` minimises it by projected gradient with Nesterov
momentum (FISTA, Beck and Teboulle 2009) and the gradient restart of
O'Donoghue and Candes (2015), step 1 / L with L the largest eigenvalue of C
over the modes.  The projection onto the constraint set is q_i =
P_i(v_i + lam), P_i the projection onto the disk of radius mu_f p_i and the
shift lam (2 components) the root of dA sum P_i(v_i + lam) = Q, found by
Newton's method.
"""
import numpy as np

from . import contact as oc
from . import elastic


def tangential_compliance_symbol(grid, E, nu):
    """C[a][b] on the full (ny, nx) DFT grid: shape (2, 2, ny, nx), 0 at k = 0."""
    nx, ny = grid['nx'], grid['ny']
    k1 = np.fft.fftfreq(nx, d=1.0 / nx) * 2 * np.pi / grid['lx']
    k2 = np.fft.fftfreq(ny, d=1.0 / ny) * 2 * np.pi / grid['ly']
    K1, K2 = np.meshgrid(k1, k2)
    q = np.hypot(K1, K2)
    nz = q > 0
    n1 = np.where(nz, K1 / np.where(nz, q, 1.0), 0.0)
    n2 = np.where(nz, K2 / np.where(nz, q, 1.0), 0.0)
    # Nyquist lines: the replicas of opposite sign average n1 n2 to zero
    nyq = np.zeros((ny, nx), dtype=bool)
    if nx % 2 == 0:
        nyq[:, nx // 2] = True
    if ny % 2 == 0:
        nyq[ny // 2, :] = True
    f = np.where(nz, 2.0 * (1.0 + nu) / (E * np.where(nz, q, 1.0)), 0.0)
    C = np.zeros((2, 2, ny, nx))
    C[0, 0] = f * (1.0 - nu * n1 * n1)
    C[1, 1] = f * (1.0 - nu * n2 * n2)
    C[0, 1] = C[1, 0] = np.where(nyq, 0.0, -f * nu * n1 * n2)
    return C


def apply_tangential(q, C):
    """u_t = C[q] for q of shape (2, ny, nx)."""
    qh = np.fft.fft2(q, axes=(1, 2))
    uh = np.einsum('abyx,byx->ayx', C, qh)
    return np.real(np.fft.ifft2(uh, axes=(1, 2)))


def coupling_symbol(grid, E, nu):
    """K[a] (a = 0, 1) on the full (ny, nx) DFT grid, complex: the
    tangential surface displacement from a normal traction t3 is
    u_a = K_a t3 per mode, and the normal surface displacement from a
    tangential traction is u3 = sum_a conj(K_a) t_a (reciprocity makes the
    3 x 3 surface compliance Hermitian per mode).  K_a = i (1 - 2 nu) n_a /
    (2 mu |k|), n = k / |k|: a compressive pressure pulls the surface towards
    itself (in plane strain d u_1 / d x_1 = -(1 + nu)(1 - 2 nu) p / E at the
    surface).  0 at k = 0 and on the Nyquist line of axis a, where the two
    replicas of opposite k_a cancel."""
    nx, ny = grid['nx'], grid['ny']
    k1 = np.fft.fftfreq(nx, d=1.0 / nx) * 2 * np.pi / grid['lx']
    k2 = np.fft.fftfreq(ny, d=1.0 / ny) * 2 * np.pi / grid['ly']
    K1, K2 = np.meshgrid(k1, k2)
    q = np.hypot(K1, K2)
    nz = q > 0
    qs = np.where(nz, q, 1.0)
    mu = E / (2.0 * (1.0 + nu))
    c = np.where(nz, (1.0 - 2.0 * nu) / (2.0 * mu * qs), 0.0)
    K = np.zeros((2, ny, nx), dtype=complex)
    K[0] = 1j * c * K1 / qs
    K[1] = 1j * c * K2 / qs
    if nx % 2 == 0:
        K[0][:, nx // 2] = 0.0
    if ny % 2 == 0:
        K[1][ny // 2, :] = 0.0
    return K


def tangential_from_normal(p, K):
    """u_t (2, ny, nx): the tangential surface displacement of the normal
    traction p (ny, nx)."""
    ph = np.fft.fft2(p)
    return np.real(np.fft.ifft2(K * ph[None], axes=(1, 2)))


def normal_from_tangential(q, K):
    """u3 (ny, nx): the normal surface displacement of the tangential
    traction q (2, ny, nx)."""
    qh = np.fft.fft2(q, axes=(1, 2))
    return np.real(np.fft.ifft2(np.conj(K[0]) * qh[0] + np.conj(K[1]) * qh[1]))


def _disk(w, rho):
    """Projection of w (2, n) onto the disks |.| <= rho (n) and its Jacobian
    sums: returns (P, sum of the 2x2 Jacobians)."""
    r = np.hypot(w[0], w[1])
    out = r > rho
    s = np.where(out, rho / np.where(out, r, 1.0), 1.0)
    P = w * s
    # Jacobian: I inside; (rho / r) (I - w w^T / r^2) outside
    with np.errstate(invalid="ignore", divide="ignore"):
        a = np.where(out, s / np.where(out, r * r, 1.0), 0.0)
    J = np.array([[np.sum(s - a * w[0] * w[0]), -np.sum(a * w[0] * w[1])],
                  [-np.sum(a * w[0] * w[1]), np.sum(s - a * w[1] * w[1])]])
    return P, J


def project(v, rho, S, lam0=None, tol=1e-15, max_iter=100):
    """argmin |q - v| over |q_i| <= rho_i, sum q = S.  v: (2, n), rho: (n),
    S: (2,).  Returns (q, lam)."""
    lam = np.zeros(2) if lam0 is None else np.array(lam0, dtype=float)
    scale = max(np.sum(rho), 1e-300)
    for _ in range(max_iter):
        P, J = _disk(v + lam[:, None], rho)
        g = P.sum(axis=1) - S
        if np.max(np.abs(g)) <= tol * scale:
            break
        J = J + 1e-14 * (np.trace(J) + 1.0) * np.eye(2)
        lam = lam - np.linalg.solve(J, g)
    P, _ = _disk(v + lam[:, None], rho)
    return P, lam


def tangential_solve(grid, E, nu, p, Q, mu_f, tol=1e-13, max_iter=100000, u0=None, q0=None):
    """Partial-slip tangential traction under the normal pressure p ((ny, nx),
    >= 0) for the total tangential force Q = (Qx, Qy) with |Q| < mu_f W.

    u0 (2, ny, nx), optional: a tangential surface displacement from other
    loads (the pressure's, with the Cerruti cross terms), added to C[q]; the
    minimised energy gains <q, u0>.  q0, optional: start from the projection
    of q0 onto the constraint set instead of the full-slip field.

    Returns (q, info): q (2, ny, nx); info with iters, the rigid shift delta
    (the stick-zone tangential displacement) and the stick fraction of the
    contact points.  Stops when dA sum |q_k - q_(k-1)| / (mu_f W) < tol."""
    nx, ny = grid['nx'], grid['ny']
    n = nx * ny
    dA = grid['lx'] * grid['ly'] / n
    p = np.asarray(p, dtype=float)
    rho = (mu_f * p).ravel()
    W = dA * p.sum()
    Q = np.asarray(Q, dtype=float)
    if not np.hypot(Q[0], Q[1]) < mu_f * W:
        raise ValueError("partial slip needs |Q| < mu_f W")
    C = tangential_compliance_symbol(grid, E, nu)
    L = float(np.max(C[0, 0] + C[1, 1]) / 2 + np.max(np.sqrt(((C[0, 0] - C[1, 1]) / 2) ** 2 + C[0, 1] ** 2)))
    S = Q / dA
    ue = np.zeros((2, n)) if u0 is None else np.asarray(u0, dtype=float).reshape(2, n)
    if q0 is None:
        # feasible start: the full-slip field scaled to the load
        q = (rho[None, :] * Q[:, None] / (mu_f * W)) if W > 0 else np.zeros((2, n))
    else:
        q, _ = project(np.asarray(q0, dtype=float).reshape(2, n), rho, S)
    y = q.copy()
    t = 1.0
    lam = np.zeros(2)
    k = 0
    change = np.inf
    while k < max_iter:
        u = apply_tangential(y.reshape(2, ny, nx), C).reshape(2, n) + ue
        qn, lam = project(y - u / L, rho, S, lam)
        change = dA * np.sum(np.abs(qn - q)) / (mu_f * W)
        k += 1
        if np.sum((y - qn) * (qn - q)) > 0.0:      # momentum points uphill: restart
            t = 1.0
            y = qn.copy()
        else:
            tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
            y = qn + ((t - 1.0) / tn) * (qn - q)
            t = tn
        q = qn
        if change < tol:
            break
    u = apply_tangential(q.reshape(2, ny, nx), C).reshape(2, n) + ue
    qa = np.hypot(q[0], q[1])
    contact = rho > 0
    stick = contact & (qa < rho * (1 - 1e-9))
    delta = u[:, stick].mean(axis=1) if np.any(stick) else np.full(2, np.nan)
    info = {"iters": k, "change": float(change), "delta": delta,
            "stick_fraction": float(np.count_nonzero(stick) / max(np.count_nonzero(contact), 1)),
            "L": L}
    return q.reshape(2, ny, nx), info


def frictional_contact_solve(grid, E, nu, h, W, Q, mu_f, coupled=True, tol=1e-13, max_iter=200,
                             tol_contact=1e-14, tol_friction=1e-13, max_contact=5000, p0=None, q0=None):
    """Normal contact under the total load W with Coulomb friction and the
    total tangential force Q (|Q| < mu_f W): the surface traction (q, p).

    coupled=False: Goodman's approximation, the frictionless normal solve
    followed by one tangential solve under its pressure.  coupled=True: the
    Boussinesq-Cerruti cross terms are kept, so the pressure solves the
    normal problem on h - u3[q] and q the tangential problem with the extra
    displacement u_t[p]; the two solves alternate, starting from q0 (0 when
    None) and p0, each warm-started from the last, until
        dA sum |p_k - p_(k-1)| / W + dA sum |q_k - q_(k-1)| / (mu_f W) < tol
    (sums over both tangential components).

    Returns (p, q, info): p (ny, nx), q (2, ny, nx); info with the number
    of alternations, the last change and the records of the last solves."""
    nx, ny = grid['nx'], grid['ny']
    dA = grid['lx'] * grid['ly'] / (nx * ny)
    h = np.asarray(h, dtype=float)
    K = coupling_symbol(grid, E, nu) if coupled else None
    q = np.zeros((2, ny, nx)) if q0 is None else np.array(q0, dtype=float)
    p = None if p0 is None else np.array(p0, dtype=float)
    change = np.inf
    k = 0
    cinfo = finfo = None
    for k in range(1, (max_iter if coupled else 1) + 1):
        hk = h - normal_from_tangential(q, K) if coupled else h
        pn, _, cinfo = oc.contact_solve(hk, W, grid, E, nu, tol=tol_contact, max_iter=max_contact, p0=p)
        u0 = tangential_from_normal(pn, K) if coupled else None
        qn, finfo = tangential_solve(grid, E, nu, pn, Q, mu_f, tol=tol_friction, u0=u0,
                                     q0=q if (coupled and (k > 1 or q0 is not None)) else None)
        if p is not None:
            change = dA * np.sum(np.abs(pn - p)) / W + dA * np.sum(np.abs(qn - q)) / (mu_f * W)
        p, q = pn, qn
        if change < tol:
            break
    return p, q, {"iters": k, "change": float(change), "contact": cinfo, "tangential": finfo}

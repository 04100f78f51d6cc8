"""Mindlin and Boussinesq operators on the periodic layered grid (oracle).

Test infrastructure only (see ``oracle/__init__``).

What is computed (the paper's Sec. 2-3, with the readings listed in the
design notes):

* Grid: nx x ny points x_j = j L/N in-plane, nz depth nodes z_i = i Lz/(nz-1).
* In-plane DFT per depth layer (Sec. 3.1, eqn dft): w_hat(k, z) =
  (1/(nx ny)) sum_x w(x, z) exp(-2 pi i (k1 x1/L1 + k2 x2/L2)); q = 2 pi kbar.
* For every mode k != 0 (Thm 1: the mode-k coefficient of the periodic
  response is the non-periodic partial-Fourier operator at q = 2 pi kbar):
  - full-space part (eqn 2gradient): grad u_inf(z_i) =
      - sum_elements q [U02 : w g0-integral + U12 : w g1-integral]
      - (jump : w(z_i)) x e3,
    with the "+" branch for elements above z_i and "-" below it;
  - Mindlin superposition (eqn mindlin_B_U): the half-space field adds the
    Boussinesq-Cerruti response to minus the surface traction of the
    full-space field, T_inf = (C : eps_inf(0) - w(0)) . n with n = -e3;
  - an applied surface traction t adds the Boussinesq-Cerruti response to t
    (operator M of eqn operators), so both operators share that last step.
* k = 0 (Remark on the fundamental mode): the laterally uniform problem,
  solved exactly: sigma.e3 = -t_mean everywhere, eps13 = (w13 - t1)/(2 mu),
  eps23 = (w23 - t2)/(2 mu), eps33 = (w33 - t3)/(lambda + 2 mu), the other
  strains 0; the displacement of this mode is set to 0.  With
  k0_policy = "exclude" the mean traction is dropped from this mode.
* Nyquist bins of even grids (k_j = N_j/2): the response is the average of
  the evaluations at q_j = +pi N_j/L_j and -pi N_j/L_j.
* Outputs are one-sided limits from inside [0, Lz]; w is zero below Lz.
"""
import numpy as np

from . import elastic
from . import fundamental as fs
from .depth import depth_sum, element_matrices


def depth_nodes(nz, lz):
    return np.linspace(0.0, lz, nz)


def grid_nodes(grid):
    """The grid's depth nodes: grid['z'] when given (Sec. 3.1 leaves the
    spacing free), else uniform on [0, lz]."""
    if grid.get('z') is not None:
        z = np.asarray(grid['z'], dtype=float)
        assert z.shape == (grid['nz'],) and z[0] == 0.0 and np.all(np.diff(z) > 0)
        return z
    return depth_nodes(grid['nz'], grid['lz'])


def sym_grad(g):
    return 0.5 * (g + np.swapaxes(g, -1, -2))


def hooke_full(eps, lam, mu):
    tr = np.trace(eps, axis1=-2, axis2=-1)
    return lam * tr[..., None, None] * np.eye(3) + 2.0 * mu * eps


def mode_response(q1, q2, w_hat, t_hat, z, E, nu, sums="dense"):
    """Per-mode response for modes with q != 0.

    sums: "dense" forms the O(N3^2) element-pair matrices (the paper's naive
    count); "recurrence" takes the same sums by depth.depth_sum in O(N3)
    (the oracle-fast mode).

    q1, q2: (M,) wavevectors; w_hat: (M, nz, 3, 3) eigenstress coefficients
    (symmetric); t_hat: (M, 3) surface traction coefficients (force per area
    exerted on the body, +e3 points into the body).  Returns grad u
    (M, nz, 3, 3) with [a, d] = d u_a / d x_d, and u (M, nz, 3).
    """
    lam, mu = elastic.lame(E, nu)
    q, grads = fs.kelvin_gradients(q1, q2, mu, nu)
    jump = fs.kelvin_jump(q1, q2, mu, nu)
    _, b00, b10, b01, b11 = fs.boussinesq_gradient(q1, q2, mu, nu)
    if sums == "dense":
        d0p, d1p, d0m, d1m = element_matrices(q, z)
        D = {('+', 0): d0p, ('+', 1): d1p, ('-', 0): d0m, ('-', 1): d1m}

        def dsum(br, k, c):
            return np.einsum('mij,mj...->mi...', D[(br, k)], c)
    else:
        def dsum(br, k, c):
            return depth_sum(q, z, c, br, k)

    # full-space part: displacement (n = 1) and its gradient (n = 2)
    grad_u = np.zeros(w_hat.shape, dtype=complex)
    u = np.zeros(w_hat.shape[:2] + (3,), dtype=complex)
    for br in ('+', '-'):
        u01, u11 = grads[(br, 1)]
        u02, u12 = grads[(br, 2)]
        for k, t1, t2 in ((0, u01, u02), (1, u11, u12)):
            c1 = np.einsum('mabc,mjbc->mja', t1, w_hat)
            c2 = np.einsum('mabcd,mjbc->mjad', t2, w_hat)
            u -= dsum(br, k, c1)
            grad_u -= q[:, None, None, None] * dsum(br, k, c2)
    grad_u[..., :, 2] -= np.einsum('mabc,mibc->mia', jump, w_hat)

    # surface traction of the full-space field, and what the half-space adds
    eps0 = sym_grad(grad_u[:, 0])
    sig0 = hooke_full(eps0, lam, mu) - w_hat[:, 0]
    t_inf = -sig0[:, :, 2]
    tau = t_hat - t_inf

    qz = q[:, None] * z[None, :]
    g0 = np.exp(-qz)
    g1 = qz * g0
    gradb = b01[:, None] * g0[..., None, None, None] + b11[:, None] * g1[..., None, None, None]
    bz = b00[:, None] * g0[..., None, None] + b10[:, None] * g1[..., None, None]
    grad_u = grad_u + np.einsum('mk,mikjl->mijl', tau, gradb)
    u = u + np.einsum('mk,mikj->mij', tau, bz) / q[:, None, None]
    return grad_u, u


def _signed(k, n):
    return k - n if k > n // 2 else k


def mode_rows(ky, kx, nx, ny, lx, ly):
    """Evaluations of bin (ky, kx) != (0, 0): (ky, kx, q1, q2, weight), once
    per sign of a Nyquist component of an even grid (weights 1/2 or 1/4)."""
    k1, k2 = _signed(kx, nx), _signed(ky, ny)
    s1 = (1, -1) if (nx % 2 == 0 and kx == nx // 2) else (1,)
    s2 = (1, -1) if (ny % 2 == 0 and ky == ny // 2) else (1,)
    wgt = 1.0 / (len(s1) * len(s2))
    return [(ky, kx, 2 * np.pi * a * k1 / lx, 2 * np.pi * b * k2 / ly, wgt) for a in s1 for b in s2]


def mode_table(nx, ny, lx, ly):
    """Evaluation list: mode_rows of every bin but k = 0."""
    rows = []
    for ky in range(ny):
        for kx in range(nx):
            if kx == 0 and ky == 0:
                continue
            rows.extend(mode_rows(ky, kx, nx, ny, lx, ly))
    return rows


def sampled_dft(f, modes):
    """DFT coefficients (1/(nx ny)) sum_x f(x) exp(-2 pi i (kx x / nx +
    ky y / ny)) over the last two axes of the real array f, at the (ky, kx)
    bins of modes (eqn dft written out; the phases are reduced exactly, as
    integers modulo n, before the trigonometric functions).  Returns shape
    f.shape[:-2] + (len(modes),)."""
    ny, nx = f.shape[-2:]
    ky = np.array([m[0] for m in modes], dtype=np.int64)
    kx = np.array([m[1] for m in modes], dtype=np.int64)
    ax = 2 * np.pi * ((kx[:, None] * np.arange(nx)[None, :]) % nx) / nx     # (M, nx)
    ay = 2 * np.pi * ((ky[:, None] * np.arange(ny)[None, :]) % ny) / ny     # (M, ny)
    F = np.ascontiguousarray(f, dtype=float).reshape(-1, nx)                # (P ny, nx)
    xr = (F @ np.cos(ax).T).reshape(-1, ny, len(modes))                     # sum_x f cos
    xi = -(F @ np.sin(ax).T).reshape(-1, ny, len(modes))                    # -sum_x f sin
    cy, sy = np.cos(ay).T, np.sin(ay).T                                     # (ny, M)
    re = np.einsum('pym,ym->pm', xr, cy) + np.einsum('pym,ym->pm', xi, sy)
    im = np.einsum('pym,ym->pm', xi, cy) - np.einsum('pym,ym->pm', xr, sy)
    return ((re + 1j * im) / (nx * ny)).reshape(f.shape[:-2] + (len(modes),))


def apply(grid, E, nu, eps_p=None, traction=None, k0_policy="include",
          chunk=256, modes=None, direct_dft=True, sums="dense"):
    """Strain, stress, displacement and surface u3 of u = M[t] + N[C:eps_p].

    grid: dict nx, ny, nz, lx, ly, lz (and optionally z, the depth nodes).  eps_p: (6, nz, ny, nx) stored
    components or None.  traction: (3, ny, nx) or None.  Returns a dict of
    physical fields: strain (6, nz, ny, nx), stress (6, nz, ny, nx) =
    C : eps - w, disp (3, nz, ny, nx), surf_u3 (ny, nx).  With ``modes`` (a
    list of (ky, kx) bins) only those bins are computed and the spectral
    coefficients are returned instead (keys strain_hat, stress_hat,
    disp_hat, each (len(modes), nz, ...)); their input coefficients come
    from sampled_dft, or with direct_dft=False from the full FFT of every
    plane (the full-field path restricted to those bins).  sums: the depth
    sums of mode_response ("recurrence" is the oracle-fast mode, with
    chunks of 4096 modes unless chunk is given otherwise).
    """
    if modes is not None and direct_dft:
        return apply_modes(grid, E, nu, eps_p, traction, modes, k0_policy)
    if sums != "dense" and chunk == 256:
        chunk = 4096
    nx, ny, nz = grid['nx'], grid['ny'], grid['nz']
    lx, ly, lz = grid['lx'], grid['ly'], grid['lz']
    lam, mu = elastic.lame(E, nu)
    z = grid_nodes(grid)
    if eps_p is None:
        w = np.zeros((6, nz, ny, nx))
    else:
        w = elastic.hooke(np.asarray(eps_p, dtype=float), E, nu)
    t = np.zeros((3, ny, nx)) if traction is None else np.asarray(traction, dtype=float)

    w_hat = np.fft.fft2(w, axes=(-2, -1)) / (nx * ny)        # (6, nz, ny, nx)
    t_hat = np.fft.fft2(t, axes=(-2, -1)) / (nx * ny)        # (3, ny, nx)
    W = elastic.to_full(np.moveaxis(w_hat, 0, -1))           # (nz, ny, nx, 3, 3)

    if modes is None:
        rows = mode_table(nx, ny, lx, ly)
    else:
        rows = [r for (ky, kx) in modes if (ky, kx) != (0, 0) for r in mode_rows(ky, kx, nx, ny, lx, ly)]
    grad = np.zeros((ny, nx, nz, 3, 3), dtype=complex)
    disp = np.zeros((ny, nx, nz, 3), dtype=complex)
    for s in range(0, len(rows), chunk):
        blk = rows[s:s + chunk]
        ky = np.array([r[0] for r in blk])
        kx = np.array([r[1] for r in blk])
        q1 = np.array([r[2] for r in blk])
        q2 = np.array([r[3] for r in blk])
        wg = np.array([r[4] for r in blk])
        wm = np.moveaxis(W[:, ky, kx], 0, 1)                  # (M, nz, 3, 3)
        tm = t_hat[:, ky, kx].T                               # (M, 3)
        g, u = mode_response(q1, q2, wm, tm, z, E, nu, sums=sums)
        np.add.at(grad, (ky, kx), wg[:, None, None, None] * g)
        np.add.at(disp, (ky, kx), wg[:, None, None] * u)

    # k = 0: laterally uniform, exact
    grad[0, 0] = k0_gradient(W[:, 0, 0], t_hat[:, 0, 0], k0_policy, lam, mu)

    eps = sym_grad(grad)                                         # (ny, nx, nz, 3, 3)
    sig = hooke_full(eps, lam, mu) - np.moveaxis(W, 0, 2)
    eps_v = elastic.to_voigt(eps)                                # (ny, nx, nz, 6)
    sig_v = elastic.to_voigt(sig)
    if modes is not None:
        ky = np.array([m[0] for m in modes])
        kx = np.array([m[1] for m in modes])
        return {'strain_hat': eps_v[ky, kx], 'stress_hat': sig_v[ky, kx],
                'disp_hat': disp[ky, kx]}

    def back(f):                       # (ny, nx, nz, c) -> (c, nz, ny, nx) real
        f = np.transpose(f, (3, 2, 0, 1))
        return np.real(np.fft.ifft2(f, axes=(-2, -1)) * (nx * ny))

    out = {'strain': back(eps_v), 'stress': back(sig_v), 'disp': back(disp)}
    out['surf_u3'] = out['disp'][2, 0].copy()
    return out


def k0_gradient(w0, t0, k0_policy, lam, mu):
    """Displacement gradient of the laterally uniform mode (exact): the
    stress vector on horizontal planes equals -t everywhere and there is no
    in-plane strain.  w0: (nz, 3, 3) mean eigenstress, t0: (3,) mean traction."""
    if k0_policy != "include":
        t0 = np.zeros(3, dtype=complex)
    g0 = np.zeros(w0.shape, dtype=complex)
    # strains through grad u: d u_a/d x3 = 2 eps_a3 for a = 1, 2
    g0[:, 0, 2] = (w0[:, 0, 2] - t0[0]) / mu
    g0[:, 1, 2] = (w0[:, 1, 2] - t0[1]) / mu
    g0[:, 2, 2] = (w0[:, 2, 2] - t0[2]) / (lam + 2.0 * mu)
    return g0


def apply_modes(grid, E, nu, eps_p, traction, modes, k0_policy="include"):
    """apply() restricted to the (ky, kx) bins of modes: the spectral
    coefficients strain_hat, stress_hat (len(modes), nz, 6) and disp_hat
    (len(modes), nz, 3), with the input coefficients taken by sampled_dft
    (no full-size arrays)."""
    nx, ny, nz = grid['nx'], grid['ny'], grid['nz']
    lx, ly, lz = grid['lx'], grid['ly'], grid['lz']
    lam, mu = elastic.lame(E, nu)
    z = grid_nodes(grid)
    M = len(modes)
    if eps_p is None:
        w_hat = np.zeros((6, nz, M), dtype=complex)
    else:
        # C : eps_p commutes with the DFT (pointwise, linear)
        w_hat = elastic.hooke(sampled_dft(np.asarray(eps_p, dtype=float), modes), E, nu)
    t_hat = np.zeros((3, M), dtype=complex) if traction is None else sampled_dft(traction, modes)
    W = elastic.to_full(np.moveaxis(w_hat, 0, -1))             # (nz, M, 3, 3)
    grad = np.zeros((M, nz, 3, 3), dtype=complex)
    disp = np.zeros((M, nz, 3), dtype=complex)
    for i, (ky, kx) in enumerate(modes):
        if ky == 0 and kx == 0:
            grad[i] = k0_gradient(W[:, i], t_hat[:, i], k0_policy, lam, mu)
            continue
        rows = mode_rows(ky, kx, nx, ny, lx, ly)
        q1 = np.array([r[2] for r in rows])
        q2 = np.array([r[3] for r in rows])
        wg = np.array([r[4] for r in rows])
        wm = np.repeat(W[None, :, i], len(rows), axis=0)        # (R, nz, 3, 3)
        tm = np.repeat(t_hat[None, :, i], len(rows), axis=0)    # (R, 3)
        g, u = mode_response(q1, q2, wm, tm, z, E, nu)
        grad[i] = np.einsum('r,rzab->zab', wg, g)
        disp[i] = np.einsum('r,rza->za', wg, u)
    eps = sym_grad(grad)                                         # (M, nz, 3, 3)
    sig = hooke_full(eps, lam, mu) - np.moveaxis(W, 0, 1)
    return {'strain_hat': elastic.to_voigt(eps), 'stress_hat': elastic.to_voigt(sig), 'disp_hat': disp}


def mindlin_apply(grid, E, nu, eps_p, **kw):
    """N[C : eps_p]: strain, stress = C:eps - C:eps_p, displacement."""
    return apply(grid, E, nu, eps_p=eps_p, traction=None, **kw)


def boussinesq_apply(grid, E, nu, traction, **kw):
    """M[t]: strain, stress = C:eps, displacement."""
    return apply(grid, E, nu, eps_p=None, traction=traction, **kw)

"""Pins of the oracle's Mindlin / Boussinesq operators (CPU only).

Each test checks the oracle against something it does not compute itself:
an independent mpmath state-space solve, textbook closed forms for
sinusoidal surface loads, brute-force DFT sums, Betti reciprocity,
symmetries and exact quadrature.
"""
import numpy as np
import pytest
import mpmath as mp

from oracle import depth, elastic, operators
from ode_reference import solve_mode
from synth import filtered_eigenstrain, filtered_traction, grid_dict

E, NU = 1.0, 0.3
LAM, MU = elastic.lame(E, NU)
ESTAR = elastic.e_star(E, NU)


def _sym(g):
    return 0.5 * (g + np.swapaxes(g, -1, -2))


# --------------------------------------------------------------- per mode --
@pytest.mark.parametrize("q1,q2,nz,lz", [
    (2 * np.pi, 0.0, 5, 0.25),            # along x
    (0.0, 2 * np.pi * 3, 6, 0.25),        # along y
    (2 * np.pi * 3, -2 * np.pi * 2, 6, 0.25),
    (0.05, 0.03, 6, 0.25),                # q dz = 0.003: series branch
    (40.0, 13.0, 7, 0.5),                 # q dz = 3.5: closed-form branch
    (2 * np.pi * 0.5, 2 * np.pi * 7, 4, 0.4),
])
def test_mode_matches_state_space_ode(q1, q2, nz, lz):
    """Oracle per-mode response == exact ODE solve (different derivation)."""
    rng = np.random.default_rng(int(1000 * (q1 + 2 * q2)) % 2**31)
    z = np.linspace(0.0, lz, nz)
    wv = rng.standard_normal((nz, 6)) + 1j * rng.standard_normal((nz, 6))
    t = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    gref, uref = solve_mode(q1, q2, z, wv, t, E, NU)
    g, u = operators.mode_response(np.array([q1]), np.array([q2]),
                                   elastic.to_full(wv)[None], t[None], z, E, NU)
    assert np.linalg.norm(g[0] - gref) <= 1e-13 * np.linalg.norm(gref)
    assert np.linalg.norm(u[0] - uref) <= 1e-13 * np.linalg.norm(uref)


@pytest.mark.parametrize("q1,q2,z", [
    (2 * np.pi, 2 * np.pi * 2, [0.0, 0.01, 0.03, 0.07, 0.15, 0.25]),      # graded toward the surface
    (40.0, 13.0, [0.0, 0.002, 0.1, 0.11, 0.5]),                            # q dz on both branches
    (0.05, 0.03, [0.0, 0.3, 0.31, 0.9]),
])
def test_mode_matches_state_space_ode_non_uniform_nodes(q1, q2, z):
    """Free node spacing (Sec. 3.1): the oracle's element integrals on
    unequal elements == the exact ODE solve on the same nodes."""
    z = np.array(z)
    nz = z.size
    rng = np.random.default_rng(int(1000 * (q1 + 3 * q2)) % 2**31)
    wv = rng.standard_normal((nz, 6)) + 1j * rng.standard_normal((nz, 6))
    t = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    gref, uref = solve_mode(q1, q2, z, wv, t, E, NU)
    g, u = operators.mode_response(np.array([q1]), np.array([q2]),
                                   elastic.to_full(wv)[None], t[None], z, E, NU)
    assert np.linalg.norm(g[0] - gref) <= 1e-13 * np.linalg.norm(gref)
    assert np.linalg.norm(u[0] - uref) <= 1e-13 * np.linalg.norm(uref)


def test_grid_nodes_feed_the_full_operator():
    """apply() with grid['z'] equals the per-mode response on those nodes
    for every bin (plumbing of the node table through the transforms)."""
    from synth import grid_dict
    g = grid_dict(4, 6, 5, lz=0.4)
    g['z'] = np.array([0.0, 0.02, 0.08, 0.2, 0.4])
    rng = np.random.default_rng(9)
    eps_p = rng.standard_normal((6, 5, 6, 4))
    full = operators.apply(g, E, NU, eps_p=eps_p)['strain']
    modes = [(1, 1), (0, 2), (3, 1)]
    spec = operators.apply(g, E, NU, eps_p=eps_p, modes=modes)['strain_hat']
    fhat = np.fft.fft2(full, axes=(2, 3)) / (4 * 6)
    for m, (ky, kx) in enumerate(modes):
        assert np.allclose(spec[m].T, fhat[:, :, ky, kx], rtol=0, atol=1e-13 * np.abs(fhat).max())
    uni = operators.apply(grid_dict(4, 6, 5, lz=0.4), E, NU, eps_p=eps_p)['strain']
    assert np.linalg.norm(uni - full) > 1e-3 * np.linalg.norm(full)


def test_mode_eigenstress_only_and_traction_only_are_additive():
    rng = np.random.default_rng(7)
    z = np.linspace(0, 0.3, 7)
    w = elastic.to_full(rng.standard_normal((7, 6)) + 1j * rng.standard_normal((7, 6)))[None]
    t = (rng.standard_normal(3) + 1j * rng.standard_normal(3))[None]
    q1, q2 = np.array([9.0]), np.array([-4.0])
    ga, _ = operators.mode_response(q1, q2, w, t, z, E, NU)
    gw, _ = operators.mode_response(q1, q2, w, 0 * t, z, E, NU)
    gt, _ = operators.mode_response(q1, q2, 0 * w, t, z, E, NU)
    assert np.allclose(ga, gw + gt, rtol=0, atol=1e-14 * np.abs(ga).max())


# ------------------------------------------------- textbook surface loads --
def _sinusoid_traction(grid, k1, k2, comp):
    nx, ny = grid['nx'], grid['ny']
    x = np.arange(nx) * grid['lx'] / nx
    y = np.arange(ny) * grid['ly'] / ny
    q1, q2 = 2 * np.pi * k1 / grid['lx'], 2 * np.pi * k2 / grid['ly']
    phase = q1 * x[None, :] + q2 * y[:, None]
    t = np.zeros((3, ny, nx))
    t[comp] = np.cos(phase)
    return t, phase, np.hypot(q1, q2), np.array([q1, q2]) / np.hypot(q1, q2)


@pytest.mark.parametrize("k1,k2", [(3, 0), (0, 2), (2, 1), (-1, 3)])
def test_boussinesq_normal_sinusoid_textbook(k1, k2):
    """Pressure cos(q.x): sigma_zz = -(1+qz)e^-qz cos, sigma_nn = -(1-qz)e^-qz cos,
    sigma_nz = -qz e^-qz sin, sigma_tt = -2 nu e^-qz cos, u_z(0) = 2/(E* q) cos."""
    g = grid_dict(16, 8, 9, lz=0.5)
    t, ph, q, n = _sinusoid_traction(g, k1, k2, 2)
    out = operators.boussinesq_apply(g, E, NU, t)
    z = np.linspace(0, g['lz'], g['nz'])[:, None, None]
    ez = np.exp(-q * z)
    s = elastic.to_full(np.moveaxis(out['stress'], 0, -1))      # (nz, ny, nx, 3, 3)
    tt = np.array([-n[1], n[0]])
    s_nn = np.einsum('a,b,...ab->...', n, n, s[..., :2, :2])
    s_tt = np.einsum('a,b,...ab->...', tt, tt, s[..., :2, :2])
    s_nz = np.einsum('a,...a->...', n, s[..., :2, 2])
    tol = 1e-13
    assert np.abs(s[..., 2, 2] + (1 + q * z) * ez * np.cos(ph)).max() < tol
    assert np.abs(s_nn + (1 - q * z) * ez * np.cos(ph)).max() < tol
    assert np.abs(s_nz + q * z * ez * np.sin(ph)).max() < tol
    assert np.abs(s_tt + 2 * NU * ez * np.cos(ph)).max() < tol
    assert np.abs(out['surf_u3'] - 2.0 / (ESTAR * q) * np.cos(ph)).max() < tol / q
    # stress = C : strain for a pure traction load
    assert np.allclose(out['stress'], elastic.hooke(out['strain'], E, NU), atol=1e-14)


@pytest.mark.parametrize("k1,k2", [(2, 0), (1, 2)])
def test_boussinesq_shear_sinusoid_textbook(k1, k2):
    """Tangential tractions: in-line shear gives u_n(0) = 2/(E* q);
    cross shear is antiplane: u_t(0) = 1/(mu q), sigma_tz = -e^-qz cos,
    sigma_nt = -e^-qz sin."""
    g = grid_dict(16, 8, 7, lz=0.4)
    nx, ny = g['nx'], g['ny']
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    q1, q2 = 2 * np.pi * k1, 2 * np.pi * k2
    q = np.hypot(q1, q2)
    n = np.array([q1, q2]) / q
    tt = np.array([-n[1], n[0]])
    ph = q1 * x[None, :] + q2 * y[:, None]
    z = np.linspace(0, g['lz'], g['nz'])[:, None, None]
    # in-line shear: traction n cos(phase)
    t = np.zeros((3, ny, nx))
    t[0], t[1] = n[0] * np.cos(ph), n[1] * np.cos(ph)
    out = operators.boussinesq_apply(g, E, NU, t)
    un0 = n[0] * out['disp'][0, 0] + n[1] * out['disp'][1, 0]
    assert np.abs(un0 - 2.0 / (ESTAR * q) * np.cos(ph)).max() < 1e-13
    # cross shear: traction tt cos(phase)
    t[0], t[1] = tt[0] * np.cos(ph), tt[1] * np.cos(ph)
    out = operators.boussinesq_apply(g, E, NU, t)
    s = elastic.to_full(np.moveaxis(out['stress'], 0, -1))
    ut0 = tt[0] * out['disp'][0, 0] + tt[1] * out['disp'][1, 0]
    s_tz = np.einsum('a,...a->...', tt, s[..., :2, 2])
    s_nt = np.einsum('a,b,...ab->...', n, tt, s[..., :2, :2])
    assert np.abs(ut0 - np.cos(ph) / (MU * q)).max() < 1e-13
    assert np.abs(s_tz + np.exp(-q * z) * np.cos(ph)).max() < 1e-13
    assert np.abs(s_nt + np.exp(-q * z) * np.sin(ph)).max() < 1e-13


# ------------------------------------------------------------- k = 0 -----
def test_k0_laterally_uniform_fields():
    """Uniform-in-plane eigenstrain and traction: equilibrium plus the free
    surface force sigma.e3 = -t_mean at every depth; in-plane strain is 0."""
    g = grid_dict(4, 4, 6, lz=0.3)
    rng = np.random.default_rng(11)
    prof = rng.standard_normal((6, 6))
    eps_p = np.broadcast_to(prof[:, :, None, None], (6, 6, 4, 4)).copy()
    tm = rng.standard_normal(3)
    t = np.broadcast_to(tm[:, None, None], (3, 4, 4)).copy()
    out = operators.apply(g, E, NU, eps_p=eps_p, traction=t)
    s = out['stress']
    assert np.abs(s[2] + tm[2]).max() < 1e-13          # sigma33
    assert np.abs(s[4] + tm[0]).max() < 1e-13          # sigma13
    assert np.abs(s[3] + tm[1]).max() < 1e-13          # sigma23
    for c in (0, 1, 5):
        assert np.abs(out['strain'][c]).max() < 1e-14
    out_x = operators.apply(g, E, NU, eps_p=eps_p, traction=t, k0_policy="exclude")
    assert np.abs(out_x['stress'][2]).max() < 1e-13 and np.abs(out_x['stress'][4]).max() < 1e-13


# ------------------------------------------------------ brute-force DFT --
def _brute_force(g, eps_p, t):
    """Explicit DFT sums + independent ODE per mode (mean-free inputs)."""
    nx, ny, nz = g['nx'], g['ny'], g['nz']
    z = np.linspace(0, g['lz'], nz)
    w = elastic.hooke(eps_p, E, NU)
    jx = np.arange(nx)
    jy = np.arange(ny)
    out = np.zeros((6, nz, ny, nx))
    for ky in range(ny):
        for kx in range(nx):
            if kx == 0 and ky == 0:
                continue
            ph = np.exp(-2j * np.pi * (kx * jx[None, :] / nx + ky * jy[:, None] / ny))
            what = np.einsum('czyx,yx->zc', w, ph) / (nx * ny)
            that = np.einsum('cyx,yx->c', t, ph) / (nx * ny)
            k1 = kx - nx if kx > nx // 2 else kx
            k2 = ky - ny if ky > ny // 2 else ky
            s1 = (1, -1) if kx == nx // 2 else (1,)
            s2 = (1, -1) if ky == ny // 2 else (1,)
            grad = 0
            for a in s1:
                for b in s2:
                    gg, _ = solve_mode(2 * np.pi * a * k1 / g['lx'], 2 * np.pi * b * k2 / g['ly'],
                                       z, what, that, E, NU, dps=30)
                    grad = grad + gg / (len(s1) * len(s2))
            eps = elastic.to_voigt(_sym(grad))                        # (nz, 6)
            back = np.exp(2j * np.pi * (kx * jx[None, :] / nx + ky * jy[:, None] / ny))
            out += np.real(np.einsum('zc,yx->czyx', eps, back))
    return out


@pytest.mark.slow
def test_brute_force_dft_tiny_grid():
    g = grid_dict(4, 4, 4, lz=0.3)
    rng = np.random.default_rng(5)
    eps_p = rng.standard_normal((6, 4, 4, 4))
    eps_p -= eps_p.mean(axis=(2, 3), keepdims=True)
    t = rng.standard_normal((3, 4, 4))
    t -= t.mean(axis=(1, 2), keepdims=True)
    ref = _brute_force(g, eps_p, t)
    out = operators.apply(g, E, NU, eps_p=eps_p, traction=t)['strain']
    assert np.linalg.norm(out - ref) <= 1e-13 * np.linalg.norm(ref)


# ----------------------------------------------------------- reciprocity --
def test_betti_reciprocity_per_mode():
    """p(-q) . u_N(q, 0) == int_0^Lz eps_M[p](-q, z) : w_h(q, z) dz.

    The right-hand side is integrated with 24-point Gauss-Legendre rules per
    element, evaluating the Boussinesq strain at the quadrature depths."""
    rng = np.random.default_rng(3)
    nz, lz = 6, 0.3
    z = np.linspace(0, lz, nz)
    q1, q2 = 17.0, -6.0
    wv = rng.standard_normal((nz, 6)) + 1j * rng.standard_normal((nz, 6))
    W = elastic.to_full(wv)
    p = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    _, uN = operators.mode_response(np.array([q1]), np.array([q2]), W[None],
                                    np.zeros((1, 3), complex), z, E, NU)
    lhs = p @ uN[0, 0]
    xg, wg = np.polynomial.legendre.leggauss(24)
    rhs = 0
    for e in range(nz - 1):
        a, b = z[e], z[e + 1]
        zs = 0.5 * (a + b) + 0.5 * (b - a) * xg
        gM, _ = operators.mode_response(np.array([-q1]), np.array([-q2]),
                                        np.zeros((1, zs.size, 3, 3), complex), p[None], zs, E, NU)
        epsM = _sym(gM[0])
        lam_ = (zs - a) / (b - a)
        wh = (1 - lam_)[:, None, None] * W[e] + lam_[:, None, None] * W[e + 1]
        rhs += 0.5 * (b - a) * np.sum(wg * np.einsum('zab,zab->z', epsM, wh))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------ symmetries --
def _rand_inputs(g, seed):
    rng = np.random.default_rng(seed)
    eps_p = rng.standard_normal((6, g['nz'], g['ny'], g['nx']))
    t = rng.standard_normal((3, g['ny'], g['nx']))
    return eps_p, t


def test_translation_invariance():
    g = grid_dict(8, 8, 5, lz=0.2)
    eps_p, t = _rand_inputs(g, 21)
    a = operators.apply(g, E, NU, eps_p=eps_p, traction=t)['strain']
    b = operators.apply(g, E, NU, eps_p=np.roll(eps_p, (1, 2), axis=(2, 3)),
                        traction=np.roll(t, (1, 2), axis=(1, 2)))['strain']
    assert np.abs(np.roll(a, (1, 2), axis=(2, 3)) - b).max() < 1e-12 * np.abs(a).max()


def test_mirror_x_symmetry():
    """x1 -> -x1 flips the sign of components with one index 1."""
    g = grid_dict(8, 8, 5, lz=0.2)
    eps_p, t = _rand_inputs(g, 22)
    sgn6 = np.array([1, 1, 1, 1, -1, -1])[:, None, None, None]
    sgn3 = np.array([-1, 1, 1])[:, None, None]

    def flip(f):
        return np.roll(f[..., ::-1], 1, axis=-1)

    a = operators.apply(g, E, NU, eps_p=eps_p, traction=t)['strain']
    b = operators.apply(g, E, NU, eps_p=sgn6 * flip(eps_p), traction=sgn3 * flip(t))['strain']
    assert np.abs(sgn6 * flip(a) - b).max() < 1e-12 * np.abs(a).max()


def test_rotation_90_symmetry():
    """Rotation by 90 degrees about e3 on a square grid."""
    g = grid_dict(8, 8, 5, lz=0.2)
    eps_p, t = _rand_inputs(g, 23)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])

    def rot_field_tensor(f):
        F = elastic.to_full(np.moveaxis(f, 0, -1))                  # (nz, ny, nx, 3, 3)
        F = np.einsum('ia,jb,...ab->...ij', R, R, F)
        # new(x) = R old(R^-1 x): index map (iy, ix) -> point R^T x
        F = _rotate_grid(F)
        return np.moveaxis(elastic.to_voigt(F), -1, 0)

    def rot_field_vector(v):
        V = np.einsum('ia,a...->i...', R, v)                        # (3, ny, nx)
        return np.moveaxis(_rotate_grid(np.moveaxis(V, 0, -1)[None])[0], -1, 0)

    a = operators.apply(g, E, NU, eps_p=eps_p, traction=t)['strain']
    b = operators.apply(g, E, NU, eps_p=rot_field_tensor(eps_p), traction=rot_field_vector(t))['strain']
    assert np.abs(rot_field_tensor(a) - b).max() < 1e-12 * np.abs(a).max()


def _rotate_grid(F):
    # F[..., iy, ix, ...] with grid axes at positions -4/-3 (tensor) or -3/-2
    # handled by the caller's layout: arrays are (nz, ny, nx, ...).
    ny, nx = F.shape[1], F.shape[2]
    out = np.empty_like(F)
    for iy in range(ny):
        for ix in range(nx):
            # point (ix, iy) comes from R^-1 (ix, iy) = (iy, -ix)
            out[:, iy, ix] = F[:, (-ix) % ny, iy % nx]
    return out


def test_real_input_gives_hermitian_spectrum():
    """The inverse DFT of the response has no imaginary part (Nyquist rule)."""
    g = grid_dict(8, 6, 4, lz=0.2)
    eps_p, t = _rand_inputs(g, 24)
    nx, ny = g['nx'], g['ny']
    modes = [(ky, kx) for ky in range(ny) for kx in range(nx)]
    spec = operators.apply(g, E, NU, eps_p=eps_p, traction=t, modes=modes)['strain_hat']
    S = np.zeros((ny, nx) + spec.shape[1:], dtype=complex)
    for (ky, kx), v in zip(modes, spec):
        S[ky, kx] = v
    Sm = np.conj(S[(-np.arange(ny)) % ny][:, (-np.arange(nx)) % nx])
    assert np.abs(S - Sm).max() < 1e-14 * np.abs(S).max()


def test_linearity():
    g = grid_dict(8, 4, 4, lz=0.2)
    a_e, a_t = _rand_inputs(g, 25)
    b_e, b_t = _rand_inputs(g, 26)
    fa = operators.apply(g, E, NU, eps_p=a_e, traction=a_t)['strain']
    fb = operators.apply(g, E, NU, eps_p=b_e, traction=b_t)['strain']
    fc = operators.apply(g, E, NU, eps_p=2 * a_e - b_e, traction=2 * a_t - b_t)['strain']
    assert np.abs(2 * fa - fb - fc).max() < 1e-13 * np.abs(fc).max()


# ----------------------------------------------------- element moments --
@pytest.mark.parametrize("a", [-14.5, -2.0000001, -1.9999999, -0.3, -1e-4, 0.0, 1e-3, 0.7, 1.9999, 2.0, 5.0])
def test_depth_moments_against_quadrature(a):
    m = depth.moments(np.array([a]))
    with mp.workdps(40):
        for n in range(3):
            ref = float(mp.quad(lambda t: t ** n * mp.exp(a * t), [-1, 0, 1]))
            assert abs(m[n][0] - ref) <= 4e-15 * max(1.0, abs(ref))


def test_sampled_dft_matches_fft():
    """sampled_dft is the DFT of eqn dft at the requested bins: equal to
    numpy's FFT coefficients (scaled by 1/(nx ny)) on random fields."""
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2, 3, 8, 16))
    modes = [(0, 0), (1, 0), (0, 1), (4, 8), (7, 15), (3, 5), (4, 3)]
    got = operators.sampled_dft(f, modes)
    ref = np.fft.fft2(f, axes=(-2, -1)) / (8 * 16)
    want = np.stack([ref[..., ky, kx] for (ky, kx) in modes], axis=-1)
    assert np.max(np.abs(got - want)) < 1e-14


def test_sampled_path_matches_full_path():
    """apply(modes=...) without full-size arrays gives the full path's
    spectral coefficients on the same bins (k = 0, Nyquist lines and the
    Nyquist corner included)."""
    g = grid_dict(8, 16, 5, 1.0, 2.0, 0.3)
    eps = filtered_eigenstrain(g, seed=3, decay=0.2)
    t = filtered_traction(g, seed=4)
    modes = [(0, 0), (0, 4), (8, 0), (8, 4), (3, 1), (15, 2), (8, 3), (1, 4)]
    a = operators.apply(g, 1.0, 0.3, eps_p=eps, traction=t, modes=modes)
    b = operators.apply(g, 1.0, 0.3, eps_p=eps, traction=t, modes=modes, direct_dft=False)
    for k in ("strain_hat", "stress_hat", "disp_hat"):
        assert np.max(np.abs(a[k] - b[k])) <= 1e-13 * np.max(np.abs(b[k])), k


# ---------------------------------------------------------------- oracle-fast
# The fast mode takes the same element sums by recurrences over the depth
# nodes (oracle/depth.py depth_sum); it is pinned to the dense element-pair
# matrices, which the tests above pin to the state-space solve.

@pytest.mark.parametrize("graded", [False, True])
def test_depth_sum_recurrence_equals_the_element_matrices(graded):
    from oracle.depth import depth_sum, element_matrices
    rng = np.random.default_rng(3)
    nz = 11
    z = 0.3 * (np.arange(nz) / (nz - 1)) ** (2.0 if graded else 1.0)
    q = np.array([1e-3, 0.2, 2.0, 17.0, 150.0, 900.0])
    D = dict(zip((("+", 0), ("+", 1), ("-", 0), ("-", 1)), element_matrices(q, z)))
    c = rng.standard_normal((q.size, nz, 3, 3)) + 1j * rng.standard_normal((q.size, nz, 3, 3))
    for key, mat in D.items():
        ref = np.einsum("mij,mjab->miab", mat, c)
        got = depth_sum(q, z, c, *key)
        scale = np.abs(ref).max(axis=(1, 2, 3), keepdims=True)
        assert np.max(np.abs(got - ref) / scale) <= 1e-13, key


@pytest.mark.parametrize("nx,ny,nz,lx,ly,graded", [(16, 12, 8, 1.0, 1.5, False), (9, 10, 5, 1.0, 1.0, False),
                                                   (32, 16, 12, 2.0, 1.0, True)])
def test_fast_operator_equals_dense_operator(nx, ny, nz, lx, ly, graded):
    """Every output of apply() with the recurrence sums equals the dense
    oracle's (odd and even sizes, Nyquist bins, graded nodes, k = 0)."""
    g = grid_dict(nx, ny, nz, lx, ly, 0.25)
    if graded:
        g["z"] = 0.25 * (np.arange(nz) / (nz - 1)) ** 2
    eps = filtered_eigenstrain(g, seed=nx)
    t = filtered_traction(g, seed=ny)
    a = operators.apply(g, E, NU, eps_p=eps, traction=t)
    b = operators.apply(g, E, NU, eps_p=eps, traction=t, sums="recurrence")
    for k in ("strain", "stress", "disp", "surf_u3"):
        assert np.linalg.norm(a[k] - b[k]) <= 1e-14 * np.linalg.norm(a[k]), k

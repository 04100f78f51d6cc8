"""Independent per-mode reference for the layered half-space (test helper).

Not the paper's method: this solves the boundary-value problem that the
Mindlin/Boussinesq operators represent, by a different route, in mpmath
arithmetic, so it can pin the oracle without sharing any formula with it.

For one in-plane mode exp(i q.x) the displacement u(z) and the total traction
tau(z) = (C : eps[u] - w) . e3 satisfy a first-order linear system
y' = A y + B w(z), y = (u, tau), obtained directly from
eps = sym grad u (grad = (i q1, i q2, d/dz)), sigma = C : eps - w and
div sigma = 0.  With w piecewise linear between the depth nodes the system is
integrated exactly element by element through the matrix exponential of an
augmented matrix.  The conditions are tau(0) = -t (the traction exerted on
the body at the surface, whose outward normal is -e3) and, below the last node
where w = 0, a solution that decays: y(Lz) lies in the generalised eigenspace
of A for the eigenvalue -|q|, i.e. (A + |q| I)^3 y(Lz) = 0.
"""
import mpmath as mp
import numpy as np


def _system(q1, q2, lam, mu):
    """A (6x6) and B (6x6 over stored w components) of y' = A y + B w."""
    i = mp.mpc(0, 1)
    iq = (i * q1, i * q2)

    def rhs(y, wv):
        u1, u2, u3, t1, t2, t3 = y
        w11, w22, w33, w23, w13, w12 = wv
        du1 = (t1 + w13) / mu - iq[0] * u3
        du2 = (t2 + w23) / mu - iq[1] * u3
        du3 = (t3 + w33 - lam * (iq[0] * u1 + iq[1] * u2)) / (lam + 2 * mu)
        e11 = iq[0] * u1
        e22 = iq[1] * u2
        e12 = (iq[1] * u1 + iq[0] * u2) / 2
        tr = e11 + e22 + du3
        s11 = lam * tr + 2 * mu * e11 - w11
        s22 = lam * tr + 2 * mu * e22 - w22
        s12 = 2 * mu * e12 - w12
        dt1 = -(iq[0] * s11 + iq[1] * s12)
        dt2 = -(iq[0] * s12 + iq[1] * s22)
        dt3 = -(iq[0] * t1 + iq[1] * t2)
        return [du1, du2, du3, dt1, dt2, dt3]

    A = mp.matrix(6, 6)
    B = mp.matrix(6, 6)
    zero6 = [mp.mpf(0)] * 6
    for c in range(6):
        e = [mp.mpf(0)] * 6
        e[c] = mp.mpf(1)
        ca = rhs(e, zero6)
        cb = rhs(zero6, e)
        for r in range(6):
            A[r, c] = ca[r]
            B[r, c] = cb[r]
    return A, B


def _strain(y, wv, q1, q2, lam, mu):
    i = mp.mpc(0, 1)
    u1, u2, u3, t1, t2, t3 = y
    w11, w22, w33, w23, w13, w12 = wv
    du1 = (t1 + w13) / mu - i * q1 * u3
    du2 = (t2 + w23) / mu - i * q2 * u3
    du3 = (t3 + w33 - lam * (i * q1 * u1 + i * q2 * u2)) / (lam + 2 * mu)
    u = (u1, u2, u3)
    du = (du1, du2, du3)
    g = [[i * q1 * u[a], i * q2 * u[a], du[a]] for a in range(3)]
    return g, u


def solve_mode(q1, q2, z, w, t, E, nu, dps=None):
    """grad u (nz, 3, 3) and u (nz, 3) at the nodes, as complex numpy arrays.

    w: (nz, 6) stored eigenstress components (complex) at the nodes,
    t: (3,) surface traction (complex).
    """
    q = float(np.hypot(q1, q2))
    lz = float(z[-1])
    if dps is None:
        dps = int(40 + 0.5 * q * lz)
    with mp.workdps(dps):
        q1m, q2m = mp.mpf(q1), mp.mpf(q2)
        E_, nu_ = mp.mpf(E), mp.mpf(nu)
        mu = E_ / (2 * (1 + nu_))
        lam = E_ * nu_ / ((1 + nu_) * (1 - 2 * nu_))
        A, B = _system(q1m, q2m, lam, mu)
        wm = [[mp.mpc(complex(w[n, c])) for c in range(6)] for n in range(len(z))]
        tm = [mp.mpc(complex(v)) for v in t]
        # affine chain y(z_n) = Phi_n y(0) + psi_n
        phis = [mp.eye(6)]
        psis = [mp.matrix(6, 1)]
        for e in range(len(z) - 1):
            h = mp.mpf(z[e + 1]) - mp.mpf(z[e])
            slope = [(wm[e + 1][c] - wm[e][c]) / h for c in range(6)]
            Bs = B * mp.matrix(slope)
            Bw = B * mp.matrix(wm[e])
            M = mp.matrix(8, 8)
            for r in range(6):
                for c in range(6):
                    M[r, c] = A[r, c]
                M[r, 6] = Bs[r]
                M[r, 7] = Bw[r]
            M[6, 7] = mp.mpf(1)
            X = mp.expm(M * h)
            Phi = mp.matrix(6, 6)
            psi = mp.matrix(6, 1)
            for r in range(6):
                for c in range(6):
                    Phi[r, c] = X[r, c]
                psi[r] = X[r, 7]
            phis.append(Phi * phis[-1])
            psis.append(Phi * psis[-1] + psi)
        # unknown u(0); tau(0) = -t
        y0c = mp.matrix([0, 0, 0, -tm[0], -tm[1], -tm[2]])
        P = (A + q * mp.eye(6)) ** 3
        Phi_l, psi_l = phis[-1], psis[-1]
        G = P * Phi_l
        rhs = -(P * (Phi_l * y0c + psi_l))
        Gu = mp.matrix(6, 3)
        for r in range(6):
            for c in range(3):
                Gu[r, c] = G[r, c]
        GH = Gu.transpose_conj()
        u0 = mp.lu_solve(GH * Gu, GH * rhs)
        y0 = mp.matrix([u0[0], u0[1], u0[2], -tm[0], -tm[1], -tm[2]])
        grads = np.zeros((len(z), 3, 3), dtype=complex)
        disp = np.zeros((len(z), 3), dtype=complex)
        for n in range(len(z)):
            y = phis[n] * y0 + psis[n]
            g, u = _strain([y[r] for r in range(6)], wm[n], q1m, q2m, lam, mu)
            for a in range(3):
                disp[n, a] = complex(u[a])
                for d in range(3):
                    grads[n, a, d] = complex(g[a][d])
    return grads, disp

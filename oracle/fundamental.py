"""Partial-Fourier fundamental solutions (oracle).

Test infrastructure only (see ``oracle/__init__``).

Follows Sec. 2.2 of the paper literally, for the in-plane mode exp(+i q.x):

* Table 1: b = 4(1-nu), Delta = (i q1/q, i q2/q, 0), Delta(+/-) = e3 -/+ Delta,
  U00(+/-) = (b I + Delta x Delta - e3 x e3) / (2 mu b),
  U10(-) = -Delta(-) x Delta(-) / (2 mu b),  U10(+) = Delta(+) x Delta(+) / (2 mu b),
  g0(+/-)(x) = exp(-/+ x),  g1(+/-)(x) = x exp(-/+ x).
  The Kelvin displacement for a field point at depth offset zeta = (field -
  source) is (1/q) [U00 g0(q zeta) + U10 g1(q zeta)], "+" for zeta > 0.
* eqn recurrence: grad^n U = q^(n-1) [U0n g0 + U1n g1] with
  U0n = -/+ U0(n-1) x Delta(+/-) + U1(n-1) x e3,  U1n = -/+ U1(n-1) x Delta(+/-);
  the new gradient index is appended last.
* B:fourier, eqn B:1_0: Boussinesq-Cerruti B = (1/q)[B00 g0(+) + B10 g1(+)],
  B00 = (2 I + (1-2nu) Delta(+) x Delta(-) + Delta x Delta - e3 x e3) / (2 mu),
  B10 = Delta(+) x Delta(+) / (2 mu);  row k of B is the displacement caused by
  a unit surface traction e_k.
* eqn jump: the jump of grad U across the source depth is U01(+) - U01(-).

All arrays are vectorised over a leading axis of modes.
"""
import numpy as np

E3 = np.array([0.0, 0.0, 1.0])


def delta_vectors(q1, q2):
    """Delta, Delta(+), Delta(-) of Table 1 for each mode; shapes (M, 3)."""
    q1 = np.asarray(q1, dtype=float)
    q2 = np.asarray(q2, dtype=float)
    q = np.hypot(q1, q2)
    d = np.zeros(q.shape + (3,), dtype=complex)
    d[..., 0] = 1j * q1 / q
    d[..., 1] = 1j * q2 / q
    dp = E3 - d          # Delta(+) = e3 - Delta
    dm = E3 + d          # Delta(-) = e3 + Delta
    return q, d, dp, dm


def outer(a, b):
    """Batched tensor product a x b; new indices of b appended after a's."""
    return np.einsum('m...,mj->m...j', a, b)


def kelvin_table1(q1, q2, mu, nu):
    """(q, U00p, U00m, U10p, U10m) of Table 1; tensors (M, 3, 3)."""
    q, d, dp, dm = delta_vectors(q1, q2)
    b = 4.0 * (1.0 - nu)
    eye = np.broadcast_to(np.eye(3), q.shape + (3, 3)).astype(complex)
    e3e3 = np.broadcast_to(np.outer(E3, E3), q.shape + (3, 3)).astype(complex)
    u00 = (b * eye + outer(d, d) - e3e3) / (2.0 * mu * b)
    u10p = outer(dp, dp) / (2.0 * mu * b)
    u10m = -outer(dm, dm) / (2.0 * mu * b)
    return q, u00, u00.copy(), u10p, u10m


def boussinesq_b(q1, q2, mu, nu):
    """(q, B00, B10) of eqn B:1_0; tensors (M, 3, 3), row = traction dir."""
    q, d, dp, dm = delta_vectors(q1, q2)
    eye = np.broadcast_to(np.eye(3), q.shape + (3, 3)).astype(complex)
    e3e3 = np.broadcast_to(np.outer(E3, E3), q.shape + (3, 3)).astype(complex)
    b00 = (2.0 * eye + (1.0 - 2.0 * nu) * outer(dp, dm) + outer(d, d) - e3e3) / (2.0 * mu)
    b10 = outer(dp, dp) / (2.0 * mu)
    return q, b00, b10


def gradient_step(u0, u1, dsign, sign):
    """One step of eqn recurrence for the branch with sign = +1 ('+') or -1.

    U0n = -sign * U0(n-1) x Delta(sign) + U1(n-1) x e3
    U1n = -sign * U1(n-1) x Delta(sign)
    """
    e3 = np.broadcast_to(E3, dsign.shape).astype(complex)
    u0n = -sign * outer(u0, dsign) + outer(u1, e3)
    u1n = -sign * outer(u1, dsign)
    return u0n, u1n


def kelvin_gradients(q1, q2, mu, nu):
    """First and second gradients of the Kelvin tensor, both branches.

    Returns q and a dict with keys ('+'|'-', n) -> (U0n, U1n), n = 1, 2, such
    that grad^n U(zeta) = q^(n-1) [U0n g0(q zeta) + U1n g1(q zeta)].
    """
    q, d, dp, dm = delta_vectors(q1, q2)
    _, u00p, u00m, u10p, u10m = kelvin_table1(q1, q2, mu, nu)
    out = {}
    a, b = u00p, u10p
    for n in (1, 2):
        a, b = gradient_step(a, b, dp, +1)
        out[('+', n)] = (a, b)
    a, b = u00m, u10m
    for n in (1, 2):
        a, b = gradient_step(a, b, dm, -1)
        out[('-', n)] = (a, b)
    return q, out


def boussinesq_gradient(q1, q2, mu, nu):
    """(q, B00, B10, B01, B11): grad B(z) = B01 g0(+)(qz) + B11 g1(+)(qz)."""
    q, d, dp, dm = delta_vectors(q1, q2)
    _, b00, b10 = boussinesq_b(q1, q2, mu, nu)
    b01, b11 = gradient_step(b00, b10, dp, +1)
    return q, b00, b10, b01, b11


def kelvin_jump(q1, q2, mu, nu):
    """eqn jump: U01(+) - U01(-), shape (M, 3, 3, 3)."""
    _, g = kelvin_gradients(q1, q2, mu, nu)
    return g[('+', 1)][0] - g[('-', 1)][0]

"""Exact P1 element integrals in depth (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. 3.2 of the paper: the eigenstress is interpolated in depth with
Lagrange shape functions (read here as P1, two nodes per element), and the
depth convolution reduces to integrals of g0 and g1 over each element.  With
the element centre x_c, half-length e and the change of variable
s = x_c + t e (t in [-1, 1]), eqns int_g0 / int_g1 give

    int_E g0(q(z - s)) phi_j(s) ds = g0(q(z - x_c)) G0_j
    int_E g1(q(z - s)) phi_j(s) ds = g0(q(z - x_c)) [q (z - x_c) G0_j + G1_j]
    G_k,j = e int_{-1}^{1} g_k(-q t e) phibar_j(t) dt.

Here z is the field (target) depth and s the source depth; the "+" branch
g0(+)(x) = exp(-x) is used for elements above the target (s <= z) and the
"-" branch g0(-)(x) = exp(x) for elements below it (s >= z).  Every element
of every target is integrated: there is no cutoff, so the cost is O(N3^2)
per mode (the paper's "naive" count, Sec. 3.2).

The moments M_n(a) = int_{-1}^{1} t^n exp(a t) dt are taken from their
closed forms for |a| >= 2 and from their Taylor series otherwise, so no
cancellation occurs for small q * e.

``depth_sum`` is the fast form of the same sums (the oracle-fast mode): the
kernel of each branch is exp(-q d) and d exp(-q d) in the distance d
between target and element centre, so the sum over the elements on one
side of a target follows from the sum at the neighbouring target by one
multiplication with exp(-q h) (h the node spacing) and the new element's
term -- a forward recurrence for the elements above, a backward one for
those below.  Same element integrals, same operator, O(N3) per mode; it is
checked against element_matrices on every grid of its tests.
"""
import math
import numpy as np


def moments(a):
    """M0, M1, M2 of exp(a t) on [-1, 1] for an array a."""
    a = np.asarray(a, dtype=float)
    m = [np.zeros_like(a) for _ in range(3)]
    small = np.abs(a) < 2.0
    if np.any(small):
        s = a[small]
        for n in range(3):
            acc = np.zeros_like(s)
            term = np.ones_like(s)          # a^k / k!
            for k in range(60):
                if (n + k) % 2 == 0:
                    acc = acc + term * (2.0 / (n + k + 1))
                term = term * s / (k + 1)
            m[n][small] = acc
    big = ~small
    if np.any(big):
        b = a[big]
        if np.max(np.abs(b)) > 600.0:
            raise ValueError("element too thick for q: |q e| > 600")
        sh, ch = np.sinh(b), np.cosh(b)
        m[0][big] = 2.0 * sh / b
        m[1][big] = 2.0 * (b * ch - sh) / (b * b)
        m[2][big] = 2.0 * ((b * b + 2.0) * sh - 2.0 * b * ch) / (b ** 3)
    return m


def element_matrices(q, z):
    """Depth-integration matrices for every mode in q (shape (M,)).

    Returns D0p, D1p, D0m, D1m of shape (M, nz, nz): entry [m, i, j] is the
    sum over elements on the given side of target node i of the integral of
    g0 (resp. g1) of q_m (z_i - s) against the P1 shape function of node j.
    """
    q = np.asarray(q, dtype=float)
    z = np.asarray(z, dtype=float)
    nz = z.size
    M = q.size
    d0p = np.zeros((M, nz, nz))
    d1p = np.zeros((M, nz, nz))
    d0m = np.zeros((M, nz, nz))
    d1m = np.zeros((M, nz, nz))
    idx = np.arange(nz)
    for e in range(nz - 1):
        xc = 0.5 * (z[e] + z[e + 1])
        eh = 0.5 * (z[e + 1] - z[e])
        dist = z[None, :] - xc                           # (1, nz): z_i - x_c
        for sgn, d0, d1, mask in ((+1.0, d0p, d1p, idx >= e + 1),
                                  (-1.0, d0m, d1m, idx <= e)):
            a = sgn * q * eh
            m0, m1, m2 = moments(a)
            g0 = {0: eh * 0.5 * (m0 - m1), 1: eh * 0.5 * (m0 + m1)}
            g1 = {0: -q * eh * eh * 0.5 * (m1 - m2), 1: -q * eh * eh * 0.5 * (m1 + m2)}
            # g0(+/-)(q (z_i - x_c)) on the targets this element serves, 0 elsewhere
            expo = np.where(mask[None, :], -sgn * q[:, None] * dist, -np.inf)
            pref = np.exp(expo)
            for side, node in ((0, e), (1, e + 1)):
                i0 = pref * g0[side][:, None]
                i1 = pref * (q[:, None] * dist * g0[side][:, None] + g1[side][:, None])
                d0[:, :, node] += i0
                d1[:, :, node] += i1
    return d0p, d1p, d0m, d1m


def depth_sum(q, z, c, branch, k):
    """D @ c for D = element_matrices(q, z)[(branch, k)] without forming D
    (branch "+": elements above the target, "-": below; k = 0: g0, 1: g1).

    q: (M,) wavenumbers; c: (M, nz, ...) nodal coefficients (any trailing
    shape).  Returns an array shaped like c.
    """
    q = np.asarray(q, dtype=float)
    z = np.asarray(z, dtype=float)
    c = np.asarray(c)
    nz = z.size
    M = q.size
    tail = (1,) * (c.ndim - 2)
    qb = q.reshape((M,) + tail)
    out = np.zeros(c.shape, dtype=np.result_type(c, float))
    if nz < 2:
        return out
    sgn = 1.0 if branch == "+" else -1.0
    H = np.diff(z)                                  # element lengths
    P = np.zeros((M,) + c.shape[2:], dtype=out.dtype)
    Q = np.zeros_like(P)
    B = np.zeros_like(P)
    order = range(nz - 1) if branch == "+" else range(nz - 2, -1, -1)
    mom = {}                                        # moments per distinct element length
    for e in order:
        eh = 0.5 * H[e]
        if eh not in mom:
            mom[eh] = moments(sgn * q * eh)
        m0, m1, m2 = mom[eh]
        g00, g01 = eh * 0.5 * (m0 - m1), eh * 0.5 * (m0 + m1)
        g10, g11 = -q * eh * eh * 0.5 * (m1 - m2), -q * eh * eh * 0.5 * (m1 + m2)
        A = g00.reshape((M,) + tail) * c[:, e] + g01.reshape((M,) + tail) * c[:, e + 1]
        Bn = g10.reshape((M,) + tail) * c[:, e] + g11.reshape((M,) + tail) * c[:, e + 1]
        rH = np.exp(-qb * H[e])
        rh = np.exp(-qb * eh)
        # move the running sums one element further from the targets, then
        # add element e (distance eh from the next target)
        Q = rH * (Q + H[e] * P) + eh * rh * A
        P = rH * P + rh * A
        B = rH * B + rh * Bn
        i = e + 1 if branch == "+" else e           # the target these sums now serve
        if k == 0:
            out[:, i] = P
        else:
            out[:, i] = sgn * qb * Q + B
    return out

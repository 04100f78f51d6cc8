"""Isotropic elasticity constants and symmetric-tensor storage (oracle).

Test infrastructure only (see ``oracle/__init__``).

Problem statement, Sec. 1 (eqn epsilon, eqn sigma): eps = sym grad u,
sigma = C : (eps - eps_p).  Symmetric tensors are stored as six components in
the order (11, 22, 33, 23, 13, 12) holding the *tensor* (not engineering)
shear values.  Inner products and norms are the full Frobenius ones, i.e. the
off-diagonal entries count twice.
"""
import numpy as np

VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
# Frobenius weight of each stored component
VOIGT_WEIGHT = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


def lame(E, nu):
    """Lame constants (lambda, mu) of the isotropic tensor C."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return lam, mu


def e_star(E, nu):
    """Hertz plane-strain modulus E* = E / (1 - nu^2) (Sec. 6.2)."""
    return E / (1.0 - nu * nu)


def to_full(v):
    """(..., 6) stored components -> (..., 3, 3) symmetric tensors."""
    v = np.asarray(v)
    out = np.zeros(v.shape[:-1] + (3, 3), dtype=v.dtype)
    for c, (a, b) in enumerate(VOIGT):
        out[..., a, b] = v[..., c]
        out[..., b, a] = v[..., c]
    return out


def to_voigt(t):
    """(..., 3, 3) tensors -> (..., 6) stored components of sym(t)."""
    t = np.asarray(t)
    out = np.empty(t.shape[:-2] + (6,), dtype=t.dtype)
    for c, (a, b) in enumerate(VOIGT):
        out[..., c] = 0.5 * (t[..., a, b] + t[..., b, a])
    return out


def hooke(eps, E, nu):
    """C : eps for stored components on axis 0: eps has shape (6, ...)."""
    lam, mu = lame(E, nu)
    eps = np.asarray(eps)
    tr = eps[0] + eps[1] + eps[2]
    out = 2.0 * mu * eps
    out[0] = out[0] + lam * tr
    out[1] = out[1] + lam * tr
    out[2] = out[2] + lam * tr
    return out

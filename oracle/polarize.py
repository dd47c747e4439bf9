"""Induced dipoles of isotropic point polarisabilities (oracle).

TEST INFRASTRUCTURE ONLY: imported by `tests/` and never by the GPU library
or its binding.

The paper's introduction notes that the method extends to induced dipoles,
the moments of polarizable force fields.  With polarisabilities alpha_i the
induced dipoles minimise

    U(mu_ind) = E(q, mu + mu_ind, Theta) + sum_i |mu_ind_i|^2 / (2 alpha_i),

E the periodic energy of eq. (1), here the classical-Ewald oracle.  E is a
quadratic form in the moments, so dE/dmu is affine in the dipoles and the
minimiser solves

    (diag(1/alpha) + H) mu_ind = -dE/dmu(q, mu, Theta),

H p = dE/dmu of the dipoles p alone.  With s_i = sqrt(alpha_i) and
mu_ind = s y this is the symmetric system (I + S H S) y = -S dE/dmu, which
also covers alpha_i = 0 (such atoms keep mu_ind_i = 0).

`induce_direct` assembles H column by column from the oracle's fields and
solves densely (tiny systems); `induce_cg` runs textbook conjugate gradients
on the same system, one oracle field evaluation per product.
"""
from __future__ import annotations

import numpy as np

from . import ewald


def _fields(pos, q, mu, theta, edge, eps, nthreads):
    """dE/dmu; zero dipoles stand in for none (the Ewald routine reports fields only with dipoles)."""
    if mu is None:
        mu = np.zeros((len(q), 3))
    return ewald(pos, q, mu, theta, edge=edge, eps=eps, nthreads=nthreads)["dEdmu"]


def _dipole_fields(pos, d, edge, eps, nthreads):
    """H d: dE/dmu of the dipoles d alone (no charges, no quadrupoles)."""
    n = len(pos)
    return _fields(pos, np.zeros(n), d.reshape(n, 3), None, edge, eps, nthreads).ravel()


def _scale(alpha):
    a = np.asarray(alpha, dtype=np.float64)
    if np.any(a < 0) or not np.all(np.isfinite(a)):
        raise ValueError("polarisabilities must be finite and >= 0")
    return np.repeat(np.sqrt(a), 3)


def induce_direct(pos, q, mu, theta, alpha, edge, eps=1e-12, nthreads=0):
    """Dense solve; H from 3n unit-dipole field evaluations.  Returns mu_ind [n][3]."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = len(pos)
    s = _scale(alpha)
    g0 = _fields(pos, q, mu, theta, edge, eps, nthreads).ravel()
    H = np.empty((3 * n, 3 * n))
    for j in range(3 * n):
        e = np.zeros(3 * n)
        e[j] = 1.0
        H[:, j] = _dipole_fields(pos, e, edge, eps, nthreads)
    A = np.eye(3 * n) + s[:, None] * H * s[None, :]
    y = np.linalg.solve(A, -s * g0)
    return (s * y).reshape(n, 3)


def induce_cg(pos, q, mu, theta, alpha, edge, eps=1e-10, tol=1e-10, max_iter=500, nthreads=0):
    """Conjugate gradients on (I + S H S) y = -S g0 from y = 0, stopping at |r| <= tol |b|.
    Returns (mu_ind [n][3], iterations, |r| / |b|)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = len(pos)
    s = _scale(alpha)
    b = -s * _fields(pos, q, mu, theta, edge, eps, nthreads).ravel()
    bb = float(b @ b)
    y = np.zeros(3 * n)
    if bb == 0.0:
        return y.reshape(n, 3), 0, 0.0
    r = b.copy()
    p = r.copy()
    rr = bb
    it = 0
    while it < max_iter:
        Ap = p + s * _dipole_fields(pos, s * p, edge, eps, nthreads)
        it += 1
        pAp = float(p @ Ap)
        if not pAp > 0.0:
            raise ArithmeticError("matrix not positive definite (polarisation catastrophe)")
        a = rr / pAp
        y += a * p
        r -= a * Ap
        rr_new = float(r @ r)
        if np.sqrt(rr_new / bb) <= tol:
            rr = rr_new
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return (s * y).reshape(n, 3), it, float(np.sqrt(rr / bb))


def polarisation_energy(pos, q, mu, theta, alpha, mu_ind, edge, eps=1e-12, nthreads=0):
    """U = E(q, mu + mu_ind, Theta) + sum_i |mu_ind_i|^2 / (2 alpha_i) (alpha_i = 0 terms need mu_ind_i = 0)."""
    n = len(np.asarray(q))
    mu_tot = np.asarray(mu_ind, dtype=np.float64).reshape(n, 3) + (0.0 if mu is None else np.asarray(mu).reshape(n, 3))
    e = ewald(pos, q, mu_tot, theta, edge=edge, eps=eps, grad=False, nthreads=nthreads)["energy"]
    a = np.asarray(alpha, dtype=np.float64)
    m2 = np.sum(np.asarray(mu_ind).reshape(n, 3) ** 2, axis=1)
    pol = np.where(a > 0, m2 / (2.0 * np.where(a > 0, a, 1.0)), 0.0)
    return float(e + pol.sum())

"""CPU FP64 oracle for the periodic point-multipole energy.

TEST INFRASTRUCTURE ONLY: imported by `tests/`, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.

`ewald` / `ewald_sites` wrap `ewald.c` (classical Ewald summation, the exact
tin-foil value of eq. (1) of the paper).  `brute` holds direct image sums for
tiny systems and `ankh_ref` a plain NumPy transcription of the ANKH-FMM
evaluation (Alg. 3 plus its adjoint) used for stage-level comparisons.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle_ewald.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ewald.c into liboracle_ewald.so with gcc (OpenMP, FP64)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
               os.path.join(_HERE, "ewald.c"), "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.oracle_ewald.restype = ctypes.c_int
        L.oracle_ewald.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_ewald_sites.restype = ctypes.c_int
        L.oracle_ewald_sites.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int64, i64p,
                                         dp, dp]
        L.oracle_near_field.restype = ctypes.c_int
        L.oracle_near_field.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_ewald_moments.restype = ctypes.c_int
        L.oracle_ewald_moments.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_dtensor.restype = ctypes.c_int
        L.oracle_dtensor.argtypes = [dp, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_ewald_o3.restype = ctypes.c_int
        L.oracle_ewald_o3.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_near_field_o3.restype = ctypes.c_int
        L.oracle_near_field_o3.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_int, dp, dp, dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def ewald_params(n: int, edge: float, eps: float = 1e-10, alpha: float | None = None):
    """Splitting parameter and cutoffs for a target accuracy eps.

    s = sqrt(ln(1/eps)) + 1; alpha balances the O(N^(3/2)) real and reciprocal
    costs; r_c = s/alpha; k_max = ceil(s alpha L / pi) (|m| <= k_max)."""
    s = math.sqrt(math.log(1.0 / eps)) + 1.0
    if alpha is None:
        alpha = math.sqrt(math.pi) * max(n, 1) ** (1.0 / 6.0) / edge
    rc = s / alpha
    kmax = int(math.ceil(s * alpha * edge / math.pi))
    return alpha, rc, kmax


def ewald(pos, q, mu=None, theta=None, edge=None, eps: float = 1e-10, alpha: float | None = None,
          grad: bool = True, nthreads: int = 0, rc: float | None = None, kmax: int | None = None, omega=None):
    """Classical Ewald energy (and forces -dE/dx, fields dE/dmu when grad).  omega: optional traceless
    octupoles [n][10] as (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz), used literally in
    Omega : grad grad grad."""
    pos = _c64(pos, (-1, 3))
    n = pos.shape[0]
    q = _c64(q, (n,))
    mu = _c64(mu, (n, 3))
    theta = _c64(theta, (n, 6))
    omega = _c64(omega, (n, 10))
    a, r, k = ewald_params(n, edge, eps, alpha)
    if rc is not None:
        r = rc
    if kmax is not None:
        k = kmax
    eo = np.zeros(5)
    F = np.zeros((n, 3)) if grad else None
    G = np.zeros((n, 3)) if grad else None
    rcode = lib().oracle_ewald_o3(n, _p(pos), _p(q), _p(mu), _p(theta), _p(omega), float(edge), float(a),
                                  float(r), int(k), int(nthreads), _p(eo), _p(F), _p(G))
    if rcode != 0:
        raise ValueError(f"oracle_ewald failed ({rcode})")
    out = dict(energy=float(eo[4]), e_real=float(eo[0]), e_rec=float(eo[1]), e_self=float(eo[2]),
               e_bg=float(eo[3]), alpha=a, rc=r, kmax=k)
    if grad:
        out["forces"] = F
        out["dEdmu"] = G
    return out


def ewald_moments(pos, q, mu=None, theta=None, edge=None, eps: float = 1e-10, alpha: float | None = None,
                  nthreads: int = 0):
    """dE/dq [n] and dE/dTheta [n][6] of the classical Ewald energy.  E is defined for traceless Theta,
    so dE/dTheta is the traceless part of the full-tensor derivative per stored component
    (xx, xy, xz, yy, yz, zz) = (G_xx, 2 G_xy, 2 G_xz, G_yy, 2 G_yz, G_zz): its dot product with any
    traceless change of the stored components is the change of E."""
    pos = _c64(pos, (-1, 3))
    n = pos.shape[0]
    q = _c64(q, (n,))
    mu = _c64(mu, (n, 3))
    theta = _c64(theta, (n, 6))
    a, r, k = ewald_params(n, edge, eps, alpha)
    dq = np.zeros(n)
    dth = np.zeros((n, 6))
    rcode = lib().oracle_ewald_moments(n, _p(pos), _p(q), _p(mu), _p(theta), float(edge), float(a), float(r),
                                       int(k), int(nthreads), _p(dq), _p(dth))
    if rcode != 0:
        raise ValueError(f"oracle_ewald_moments failed ({rcode})")
    return dict(dEdq=dq, dEdtheta=dth, alpha=a, rc=r, kmax=k)


def ewald_sites(pos, q, mu, theta, edge, sel, eps: float = 1e-10, alpha: float | None = None,
                nthreads: int = 0):
    """Forces and fields on the atoms `sel` only (energy not computed)."""
    pos = _c64(pos, (-1, 3))
    n = pos.shape[0]
    q = _c64(q, (n,))
    mu = _c64(mu, (n, 3))
    theta = _c64(theta, (n, 6))
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    a, r, k = ewald_params(n, edge, eps, alpha)
    F = np.zeros((len(sel), 3))
    G = np.zeros((len(sel), 3))
    rcode = lib().oracle_ewald_sites(n, _p(pos), _p(q), _p(mu), _p(theta), float(edge), float(a), float(r),
                                     int(k), int(nthreads), len(sel),
                                     sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(F), _p(G))
    if rcode != 0:
        raise ValueError(f"oracle_ewald_sites failed ({rcode})")
    return dict(forces=F, dEdmu=G, alpha=a, rc=r, kmax=k)


def dtensor(r, alpha: float, n: int) -> np.ndarray:
    """Rank-n Cartesian derivative tensor of erfc(alpha r)/r at r (3^n values)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros(3 ** n)
    if lib().oracle_dtensor(_p(r), float(alpha), int(n), _p(out)) != 0:
        raise ValueError("bad rank")
    return out.reshape((3,) * n) if n > 0 else out

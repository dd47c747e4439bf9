"""Direct image sums of eq. (1) for tiny systems (test infrastructure only).

The lattice sum of eq. (1) is only conditionally convergent; summed over
growing cubes of images |n|_inf <= P it converges, for a neutral cell with
zero dipole moment, to the tin-foil value that classical Ewald summation
returns.  For a cell with dipole M the cube limit exceeds the tin-foil value by
2 pi |M|^2 / (3 V) (a cube has the depolarisation factor of a sphere).

Only point charges are summed here: multipoles are pinned separately as
limits of charge clusters.  The truncation error of the cube sum decays as a
power series in 1/P; `cube_limit` removes the leading terms by least squares
on a range of P (Richardson-style extrapolation).
"""
from __future__ import annotations

import numpy as np


def cube_sum(pos: np.ndarray, q: np.ndarray, edge: float, P: int) -> float:
    """1/2 sum over images |n|_inf <= P of sum_ij q_i q_j / |r_i - r_j + n L| (i=j, n=0 dropped)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    d = pos[:, None, :] - pos[None, :, :]            # [n, n, 3]
    qq = q[:, None] * q[None, :]
    rng = np.arange(-P, P + 1, dtype=np.float64) * edge
    total = 0.0
    for sx in rng:
        # vectorise over the (y, z) plane of images for this x-slab
        sy, sz = np.meshgrid(rng, rng, indexing="ij")
        sh = np.stack([np.full(sy.size, sx), sy.ravel(), sz.ravel()], axis=1)   # [m, 3]
        r = d[None, :, :, :] + sh[:, None, None, :]
        dist = np.sqrt(np.sum(r * r, axis=-1))                              # [m, n, n]
        zero = dist == 0.0
        dist[zero] = 1.0
        contrib = np.where(zero, 0.0, qq[None] / dist)
        total += 0.5 * float(np.sum(contrib))
    return total


def cube_limit(pos, q, edge: float, Ps=(10, 12, 14, 16, 18, 20, 22, 24), powers=(2, 3, 4, 5, 6)) -> float:
    """Extrapolate cube_sum(P) to P -> infinity by a least-squares fit
    E(P) = E_inf + sum_k c_k / P^k over the given P values."""
    Ps = np.asarray(Ps, dtype=np.float64)
    E = np.array([cube_sum(pos, q, edge, int(P)) for P in Ps])
    A = np.stack([np.ones_like(Ps)] + [Ps ** (-k) for k in powers], axis=1)
    coef, *_ = np.linalg.lstsq(A, E, rcond=None)
    return float(coef[0])

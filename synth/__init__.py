"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module only draws random inputs; it holds none of the method's arithmetic.
Every generator returns a dict with

  pos    float64 [N, 3]   positions, wrapped into [-r_B, r_B)^3 (Angstrom)
  q      float64 [N]      charges (e)
  mu     float64 [N, 3]   dipoles (e*Angstrom) or None
  theta  float64 [N, 6]   traceless symmetric quadrupoles (e*Angstrom^2) in the
                          component order (xx, xy, xz, yy, yz, zz), or None
  edge   float            cubic box edge 2*r_B (Angstrom)
  name   str

The water boxes stand in for the water boxes the paper benchmarks on (its
numerical-results section): same density (0.0334 molecules per cubic Angstrom,
0.1 atoms per cubic Angstrom), rigid 3-site geometry, random orientations.
"""
from __future__ import annotations

import math

import numpy as np

WATER_DENSITY = 0.0334          # molecules / A^3
ROH = 0.9572                    # A
HOH_DEG = 104.52                # degrees
Q_O, Q_H = -0.834, 0.417


def _wrap(pos: np.ndarray, edge: float) -> np.ndarray:
    r = 0.5 * edge
    out = pos - edge * np.floor((pos + r) / edge)
    # guard the half-open interval against round-up to +r
    out[out >= r] -= edge
    return out


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations from normalised 4-D Gaussian quaternions."""
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_traceless_theta(rng: np.random.Generator, n: int, sigma: float) -> np.ndarray:
    """xx, yy, xy, xz, yz ~ N(0, sigma); zz = -xx - yy. Order (xx, xy, xz, yy, yz, zz)."""
    xx = rng.normal(0.0, sigma, n)
    yy = rng.normal(0.0, sigma, n)
    xy = rng.normal(0.0, sigma, n)
    xz = rng.normal(0.0, sigma, n)
    yz = rng.normal(0.0, sigma, n)
    zz = -xx - yy
    return np.stack([xx, xy, xz, yy, yz, zz], axis=1)


def random_traceless_omega(rng: np.random.Generator, n: int, sigma: float) -> np.ndarray:
    """Traceless symmetric octupoles [n][10] in the order (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz,
    zzz): xxx, xxy, xxz, xyy, xyz, yyy, yyz ~ N(0, sigma), and the three traces zero,
    xzz = -xxx - xyy, yzz = -xxy - yyy, zzz = -xxz - yyz."""
    o = np.zeros((n, 10))
    free = [0, 1, 2, 3, 4, 6, 7]
    o[:, free] = rng.normal(0.0, sigma, (n, 7))
    o[:, 5] = -o[:, 0] - o[:, 3]
    o[:, 8] = -o[:, 1] - o[:, 6]
    o[:, 9] = -o[:, 2] - o[:, 7]
    return o


def water_octupoles(n_mol: int, seed: int = 2, sigma: float = 0.05) -> np.ndarray:
    """Octupoles for a water box of n_mol molecules (3 n_mol atoms), seeded apart from the box itself."""
    return random_traceless_omega(np.random.default_rng(1000 + seed), 3 * n_mol, sigma)


def charges(n: int = 1000, edge: float = 24.0, seed: int = 1) -> dict:
    """n point charges, uniform in the box, half +1 and half -1 (neutral for even n)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-0.5 * edge, 0.5 * edge, (n, 3))
    q = -np.ones(n)
    q[rng.permutation(n)[: n // 2]] = 1.0
    return dict(pos=_wrap(pos, edge), q=q, mu=None, theta=None, edge=float(edge),
                name=f"charges_n{n}")


def water(n_mol: int, seed: int = 2, mu_sigma: float = 0.1, theta_sigma: float = 0.1,
          jitter: float = 0.1, with_mu: bool = True, with_theta: bool = True) -> dict:
    """Rigid 3-site water on a jittered cubic lattice at 0.0334 molecules/A^3.

    Sites: the smallest m^3 >= n_mol lattice; n_mol of them chosen by a seeded
    permutation; jitter uniform +-jitter*spacing per axis; uniform random
    orientation; O at the site, the two H at ROH and +-HOH/2 from the bisector.
    Atoms are ordered O, H, H per molecule.
    """
    rng = np.random.default_rng(seed)
    edge = (n_mol / WATER_DENSITY) ** (1.0 / 3.0)
    m = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    while m ** 3 < n_mol:
        m += 1
    spacing = edge / m
    sites = rng.permutation(m ** 3)[:n_mol]
    ijk = np.stack([sites // (m * m), (sites // m) % m, sites % m], axis=1).astype(np.float64)
    centres = -0.5 * edge + (ijk + 0.5) * spacing
    centres += rng.uniform(-jitter * spacing, jitter * spacing, centres.shape)
    half = math.radians(HOH_DEG) / 2.0
    body = np.array([[0.0, 0.0, 0.0],
                     [ROH * math.sin(half), 0.0, ROH * math.cos(half)],
                     [-ROH * math.sin(half), 0.0, ROH * math.cos(half)]])
    R = _random_rotations(rng, n_mol)
    atoms = centres[:, None, :] + np.einsum("mij,aj->mai", R, body)
    pos = atoms.reshape(-1, 3)
    n = pos.shape[0]
    q = np.tile(np.array([Q_O, Q_H, Q_H]), n_mol)
    mu = rng.normal(0.0, mu_sigma, (n, 3)) if with_mu else None
    theta = random_traceless_theta(rng, n, theta_sigma) if with_theta else None
    return dict(pos=_wrap(pos, edge), q=q, mu=mu, theta=theta, edge=float(edge),
                name=f"water_nmol{n_mol}")


def water_polarisabilities(n_mol: int, alpha_o: float = 0.3, alpha_h: float = 0.03) -> np.ndarray:
    """Isotropic point polarisabilities (A^3) in the atom order of `water` (O, H, H per molecule).

    The kernel has no short-range damping, so the values are kept small enough that the undamped
    dipole-dipole coupling 2 sqrt(alpha_i alpha_j) / r^3 stays below 0.25 for the O-H bond (0.957 A)
    and for the closest intermolecular H-H pairs of the seeded boxes (0.63 A): the induced-dipole
    matrix stays positive definite."""
    return np.tile(np.array([alpha_o, alpha_h, alpha_h]), n_mol)


def ionic(n: int, density: float = 0.1, seed: int = 4, mu_sigma: float = 0.05) -> dict:
    """Ionic melt: n charges +-1 (neutral), uniform at `density` atoms/A^3, N(0, mu_sigma) dipoles."""
    rng = np.random.default_rng(seed)
    edge = (n / density) ** (1.0 / 3.0)
    pos = rng.uniform(-0.5 * edge, 0.5 * edge, (n, 3))
    q = -np.ones(n)
    q[rng.permutation(n)[: n // 2]] = 1.0
    mu = rng.normal(0.0, mu_sigma, (n, 3)) if mu_sigma > 0 else None
    return dict(pos=_wrap(pos, edge), q=q, mu=mu, theta=None, edge=float(edge),
                name=f"ionic_n{n}")


def water_cutout(src: dict, sub_edge: float) -> dict:
    """Whole molecules whose O lies in the corner sub-cube of edge sub_edge,
    re-wrapped as a periodic box of that edge (neutral: molecules are whole)."""
    pos = src["pos"].reshape(-1, 3, 3)
    r = 0.5 * src["edge"]
    o = pos[:, 0, :]
    keep = np.all(o + r < sub_edge, axis=1)
    # unwrap each molecule around its O so that it stays whole
    d = pos - o[:, None, :]
    d -= src["edge"] * np.round(d / src["edge"])
    mol = (o[:, None, :] + d)[keep]
    shift = -r + 0.5 * sub_edge
    newpos = _wrap((mol - shift).reshape(-1, 3) - 0.0, sub_edge)
    idx = np.repeat(np.nonzero(keep)[0] * 3, 3) + np.tile(np.arange(3), int(keep.sum()))
    out = dict(pos=newpos, q=src["q"][idx].copy(), edge=float(sub_edge),
               mu=None if src["mu"] is None else src["mu"][idx].copy(),
               theta=None if src["theta"] is None else src["theta"][idx].copy(),
               name=src["name"] + f"_cut{sub_edge:.3f}")
    return out


def nacl_conventional(n_cells: int = 1, a: float = 2.0) -> dict:
    """Rock-salt crystal: n_cells^3 conventional cubic cells of edge a, 4 Na+ and 4 Cl- each."""
    base_na = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    base_cl = base_na + np.array([.5, 0, 0])
    pts, qs = [], []
    for i in range(n_cells):
        for j in range(n_cells):
            for k in range(n_cells):
                o = np.array([i, j, k], dtype=np.float64)
                pts.append((base_na + o) * a)
                qs.append(np.ones(4))
                pts.append((base_cl + o) * a)
                qs.append(-np.ones(4))
    edge = n_cells * a
    pos = np.concatenate(pts) - 0.5 * edge + 0.25 * a
    return dict(pos=_wrap(pos, edge), q=np.concatenate(qs), mu=None, theta=None,
                edge=float(edge), name=f"nacl_{n_cells}")


# Standard workloads, seeds 1..5 ------------------------------------------------

def workload(name: str) -> dict:
    if name == "charges_1000":
        return charges(1000, 24.0, seed=1)
    if name == "water_9000":
        return water(3000, seed=2)
    if name == "water_288000":
        return water(96000, seed=3)
    if name == "ionic_1000000":
        return ionic(1_000_000, seed=4)
    if name == "water_9000000":
        return water(3_000_000, seed=5)
    raise KeyError(name)

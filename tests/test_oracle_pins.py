"""Pins of the classical-Ewald oracle against values fixed by the mathematics.

Each test targets a different part of the oracle so that a plausible mistake
(a dropped term, a wrong sign or factor, a transposed operand) fails one of
them:

* rock-salt / CsCl Madelung constants: charge path, the 1/2 convention,
  real + reciprocal + self terms;
* one charge in a cubic box: the neutralising background term;
* one dipole per cubic cell: dipole operator sign and the tin-foil boundary;
* independence of the splitting parameter: consistency of the real,
  reciprocal and self terms for dipoles and quadrupoles;
* dipoles and quadrupoles as limits of charge clusters: the normalisation of
  mu . grad and Theta : grad grad (no 1/2 or 1/3 factor);
* brute-force cube sums on tiny cells: the summation convention of eq. (1);
* finite differences: forces -dE/dx and fields dE/dmu;
* potentials dE/dq: the rock-salt site potential -M/r0 and finite differences;
* quadrupole derivatives dE/dTheta: a point charge's field gradient and
  finite differences along traceless directions;
* derivative tensors: rank n+1 equals the gradient of rank n.
"""
import math

import numpy as np
import pytest

import synth
from oracle import brute

EPS = 1e-14


def _rand_system(seed, n=24, edge=9.0, neutral=True, with_mu=True, with_theta=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-0.5 * edge, 0.5 * edge, (n, 3))
    q = rng.normal(size=n)
    if neutral:
        q -= q.mean()
    mu = 0.3 * rng.normal(size=(n, 3)) if with_mu else None
    th = synth.random_traceless_theta(rng, n, 0.2) if with_theta else None
    return pos, q, mu, th, edge


@pytest.mark.parametrize("ncell", [1, 2])
def test_nacl_madelung(oracle_lib, ncell):
    # conventional cell of edge a = 2 (nearest-neighbour distance 1) holds 4 ion pairs:
    # E = -4 n^3 M, M = 1.747564594633 (rock salt)
    d = synth.nacl_conventional(ncell, 2.0)
    e = oracle_lib.ewald(d["pos"], d["q"], edge=d["edge"], eps=EPS, grad=False)["energy"]
    assert e == pytest.approx(-4 * ncell ** 3 * 1.747564594633, rel=1e-11)


def test_cscl_madelung(oracle_lib):
    # CsCl: ions at the corner and body centre of a cube of edge a; nearest distance a sqrt(3)/2;
    # E per ion pair = -M / r0 with M = 1.762674773
    a = 2.0
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]) * a - 0.3
    q = np.array([1.0, -1.0])
    e = oracle_lib.ewald(pos, q, edge=a, eps=EPS, grad=False)["energy"]
    r0 = a * math.sqrt(3) / 2
    assert e == pytest.approx(-1.762674773 / r0, rel=1e-9)


def test_single_charge_background(oracle_lib):
    # simple-cubic lattice of unit charges in a neutralising background:
    # E = q^2 xi_sc / (2 L) with xi_sc = -2.837297479
    for edge in (10.0, 3.7):
        for alpha in (0.3, 0.8):
            e = oracle_lib.ewald(np.zeros((1, 3)), np.ones(1), edge=edge, eps=EPS, alpha=alpha / edge * 10,
                                 grad=False)["energy"]
            assert e == pytest.approx(-2.837297479 / (2 * edge), rel=1e-9)


def test_dipole_lattice(oracle_lib):
    # one dipole per cubic cell, tin-foil boundary: E = -2 pi |mu|^2 / (3 V)
    mu = np.array([[0.3, -0.2, 0.5]])
    edge = 7.0
    e = oracle_lib.ewald(np.zeros((1, 3)), np.zeros(1), mu=mu, edge=edge, eps=EPS, grad=False)["energy"]
    assert e == pytest.approx(-2 * math.pi * np.sum(mu ** 2) / (3 * edge ** 3), rel=1e-11)


@pytest.mark.parametrize("neutral", [True, False])
def test_alpha_independence(oracle_lib, neutral):
    pos, q, mu, th, edge = _rand_system(11, neutral=neutral)
    es = []
    for a in (0.35, 0.5, 0.75):
        o = oracle_lib.ewald(pos, q, mu, th, edge=edge, eps=EPS, alpha=a, grad=False)
        es.append(o["energy"])
    es = np.array(es)
    assert np.max(np.abs(es - es[0])) <= 1e-12 * abs(es[0])


def test_translation_invariance(oracle_lib):
    pos, q, mu, th, edge = _rand_system(12)
    e0 = oracle_lib.ewald(pos, q, mu, th, edge=edge, eps=EPS, grad=False)["energy"]
    shift = np.array([1.234, -3.21, 7.7])
    e1 = oracle_lib.ewald(pos + shift, q, mu, th, edge=edge, eps=EPS, grad=False)["energy"]
    assert e1 == pytest.approx(e0, rel=1e-13)


def _subtract_intra(posc, qc, groups):
    e = 0.0
    for g in groups:
        for a in range(len(g)):
            for b in range(a + 1, len(g)):
                i, j = g[a], g[b]
                e += qc[i] * qc[j] / np.linalg.norm(posc[i] - posc[j])
    return e


def _dipole_clusters(pos, q, mu, d):
    P, Q, groups = [], [], []
    for i in range(len(q)):
        g = [len(Q)]
        P.append(pos[i]); Q.append(q[i])
        m = np.linalg.norm(mu[i])
        u = mu[i] / m
        for s in (+1, -1):
            g.append(len(Q))
            P.append(pos[i] + s * 0.5 * d * u)
            Q.append(s * m / d)
        groups.append(g)
    return np.array(P), np.array(Q), groups


def _quad_clusters(pos, q, th, d):
    P, Q, groups = [], [], []
    for i in range(len(q)):
        T = np.array([[th[i, 0], th[i, 1], th[i, 2]],
                      [th[i, 1], th[i, 3], th[i, 4]],
                      [th[i, 2], th[i, 4], th[i, 5]]])
        lam, vec = np.linalg.eigh(T)
        g = [len(Q)]
        P.append(pos[i]); Q.append(q[i])
        for k in range(3):
            for s in (+1, -1):
                g.append(len(Q))
                P.append(pos[i] + s * d * vec[:, k])
                Q.append(lam[k] / d ** 2)
        groups.append(g)
    return np.array(P), np.array(Q), groups


def _richardson(f, d, levels=2):
    # E(d) = E0 + c1 d^2 + c2 d^4 + ...: eliminate the first levels-1 even powers
    vals = [f(d / 2 ** k) for k in range(levels)]
    for j in range(1, levels):
        vals = [(4 ** j * vals[k + 1] - vals[k]) / (4 ** j - 1) for k in range(len(vals) - 1)]
    return vals[0]


def test_dipole_is_charge_pair_limit(oracle_lib):
    pos, q, mu, _, edge = _rand_system(13, n=6, with_theta=False)
    ref = oracle_lib.ewald(pos, q, mu, None, edge=edge, eps=EPS, grad=False)["energy"]

    def e_of(d):
        P, Q, groups = _dipole_clusters(pos, q, mu, d)
        e = oracle_lib.ewald(P, Q, edge=edge, eps=EPS, alpha=0.5, grad=False)["energy"]
        return e - _subtract_intra(P, Q, groups)

    est = _richardson(e_of, 0.02)
    assert est == pytest.approx(ref, rel=2e-8)


def test_quadrupole_is_charge_cluster_limit(oracle_lib):
    pos, q, _, th, edge = _rand_system(14, n=5, with_mu=False)
    ref = oracle_lib.ewald(pos, q, None, th, edge=edge, eps=EPS, grad=False)["energy"]

    def e_of(d):
        P, Q, groups = _quad_clusters(pos, q, th, d)
        e = oracle_lib.ewald(P, Q, edge=edge, eps=EPS, alpha=0.5, grad=False)["energy"]
        return e - _subtract_intra(P, Q, groups)

    # a wrong normalisation (a 1/2 or 1/3 factor) would be an O(1) error
    est = _richardson(e_of, 0.08, levels=3)
    assert est == pytest.approx(ref, rel=1e-6)


def test_brute_cube_sum_neutral_symmetric(oracle_lib):
    # inversion-symmetric neutral cell: zero dipole, cube limit = tin-foil value
    rng = np.random.default_rng(5)
    h = rng.uniform(-2, 2, (3, 3))
    qh = np.array([1.0, -0.6, -0.4])
    pos = np.concatenate([h, -h])
    q = np.concatenate([qh, qh])
    e = oracle_lib.ewald(pos, q, edge=5.0, eps=EPS, grad=False)["energy"]
    assert brute.cube_limit(pos, q, 5.0) == pytest.approx(e, rel=1e-10)


def test_brute_cube_sum_with_dipole_moment(oracle_lib):
    rng = np.random.default_rng(6)
    pos = rng.uniform(-2, 2, (4, 3))
    q = np.array([1.0, -1.0, 0.5, -0.5])
    M = (q[:, None] * pos).sum(0)
    edge = 5.0
    e = oracle_lib.ewald(pos, q, edge=edge, eps=EPS, grad=False)["energy"]
    cube = brute.cube_limit(pos, q, edge)
    assert cube == pytest.approx(e + 2 * math.pi * np.sum(M ** 2) / (3 * edge ** 3), rel=1e-10)


def test_forces_fields_finite_difference(oracle_lib):
    pos, q, mu, th, edge = _rand_system(15, n=16)
    o = oracle_lib.ewald(pos, q, mu, th, edge=edge, eps=EPS, alpha=0.45)
    h = 1e-5
    for i in (0, 7):
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, d] += h
            p2[i, d] -= h
            e1 = oracle_lib.ewald(p1, q, mu, th, edge=edge, eps=EPS, alpha=0.45, grad=False)["energy"]
            e2 = oracle_lib.ewald(p2, q, mu, th, edge=edge, eps=EPS, alpha=0.45, grad=False)["energy"]
            assert -(e1 - e2) / (2 * h) == pytest.approx(o["forces"][i, d], rel=1e-7, abs=1e-9)
            m1, m2 = mu.copy(), mu.copy()
            m1[i, d] += h
            m2[i, d] -= h
            e1 = oracle_lib.ewald(pos, q, m1, th, edge=edge, eps=EPS, alpha=0.45, grad=False)["energy"]
            e2 = oracle_lib.ewald(pos, q, m2, th, edge=edge, eps=EPS, alpha=0.45, grad=False)["energy"]
            assert (e1 - e2) / (2 * h) == pytest.approx(o["dEdmu"][i, d], rel=1e-7, abs=1e-9)


def test_potential_rock_salt_site(oracle_lib):
    # every site of a rock-salt crystal sits at potential -q_i M / r0 (r0 = 1: nearest neighbours)
    d = synth.nacl_conventional(2, 2.0)
    m = oracle_lib.ewald_moments(d["pos"], d["q"], edge=d["edge"], eps=EPS)
    np.testing.assert_allclose(m["dEdq"], -d["q"] * 1.747564594633, rtol=1e-11)


def test_field_gradient_of_a_point_charge(oracle_lib):
    # a charge q at the origin and a bare quadrupole at r z in a box much larger than r: dE/dTheta is
    # q d_a d_b (1/r) = q (3 r_a r_b - r^2 delta_ab) / r^5, per stored component (xy, xz, yz doubled);
    # the images and the background add an isotropic part (removed with the trace) and
    # anisotropic parts of relative size (r / L)^3
    L, r, qc = 200.0, 2.5, 0.7
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    th = np.zeros((2, 6))
    th[1] = [0.1, 0.05, -0.02, 0.2, 0.03, -0.3]
    m = oracle_lib.ewald_moments(pos, np.array([qc, 0.0]), None, th, edge=L, eps=EPS)
    c = qc / r ** 3
    np.testing.assert_allclose(m["dEdtheta"][1], [-c, 0, 0, -c, 0, 2 * c], rtol=1e-5, atol=1e-6 * c)


def test_moment_derivatives_finite_difference(oracle_lib):
    pos, q, mu, th, edge = _rand_system(19, n=16)
    m = oracle_lib.ewald_moments(pos, q, mu, th, edge=edge, eps=EPS, alpha=0.45)
    E = lambda q_, th_: oracle_lib.ewald(pos, q_, mu, th_, edge=edge, eps=EPS, alpha=0.45, grad=False)["energy"]
    h = 1e-5
    for i in (0, 9):
        q1, q2 = q.copy(), q.copy()
        q1[i] += h
        q2[i] -= h
        assert (E(q1, th) - E(q2, th)) / (2 * h) == pytest.approx(m["dEdq"][i], rel=1e-7, abs=1e-9)
        # traceless directions of the stored components
        for dl in ([0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0], [0, 0, 0, 0, 1, 0], [1, 0, 0, -1, 0, 0],
                   [1, 0, 0, 0, 0, -1]):
            dl = np.array(dl, dtype=np.float64)
            t1, t2 = th.copy(), th.copy()
            t1[i] += h * dl
            t2[i] -= h * dl
            assert (E(q, t1) - E(q, t2)) / (2 * h) == pytest.approx(m["dEdtheta"][i] @ dl, rel=1e-7, abs=1e-9)
    # the reported derivative is traceless
    np.testing.assert_allclose(m["dEdtheta"][:, 0] + m["dEdtheta"][:, 3] + m["dEdtheta"][:, 5], 0, atol=1e-12)


def test_sites_match_full(oracle_lib):
    pos, q, mu, th, edge = _rand_system(16, n=30)
    full = oracle_lib.ewald(pos, q, mu, th, edge=edge, eps=EPS)
    sel = np.array([3, 17, 29])
    part = oracle_lib.ewald_sites(pos, q, mu, th, edge, sel, eps=EPS)
    np.testing.assert_allclose(part["forces"], full["forces"][sel], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(part["dEdmu"], full["dEdmu"][sel], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_derivative_tensors(oracle_lib, n):
    r = np.array([0.7, -0.4, 1.1])
    a = 0.6
    h = 1e-5
    Tn = oracle_lib.dtensor(r, a, n)
    for e in range(3):
        rp, rm = r.copy(), r.copy()
        rp[e] += h
        rm[e] -= h
        fd = (oracle_lib.dtensor(rp, a, n - 1) - oracle_lib.dtensor(rm, a, n - 1)) / (2 * h)
        np.testing.assert_allclose(Tn[..., e], fd, rtol=1e-6, atol=1e-8)
    # symmetric in all indices
    if n >= 2:
        np.testing.assert_allclose(Tn, np.swapaxes(Tn, 0, 1), rtol=1e-14, atol=1e-15)
    # traceless away from the origin for the pure 1/r part is not expected for erfc; check the
    # zero-alpha limit instead: T_ab of 1/r is (3 r_a r_b - r^2 delta_ab)/r^5
    if n == 2:
        T = oracle_lib.dtensor(r, 1e-9, 2)
        r2 = r @ r
        ref = (3 * np.outer(r, r) - r2 * np.eye(3)) / r2 ** 2.5
        np.testing.assert_allclose(T, ref, rtol=1e-7)


# ---- octupoles (the next multipole order of the operator D) ------------------------------------------

def _octupole_system(seed, n=24, edge=9.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-0.5 * edge, 0.5 * edge, (n, 3))
    q = rng.normal(0.0, 0.5, n)
    q -= q.mean()
    mu = rng.normal(0.0, 0.2, (n, 3))
    th = synth.random_traceless_theta(rng, n, 0.2)
    om = synth.random_traceless_omega(rng, n, 0.2)
    return pos, q, mu, th, om, edge


def test_octupole_alpha_independence():
    """The splitting parameter cancels exactly with octupoles present: the reciprocal factor -i Omega:kkk
    and the self term 48 a^6/7 Omega:Omega balance the real-space octupole terms (energy, forces, fields)."""
    import oracle
    pos, q, mu, th, om, L = _octupole_system(5)
    a0 = oracle.ewald_params(len(q), L, 1e-14)[0]
    res = [oracle.ewald(pos, q, mu, th, edge=L, eps=1e-14, alpha=f * a0, omega=om) for f in (0.75, 1.0, 1.5)]
    E = [r["energy"] for r in res]
    assert max(abs(e - E[1]) for e in E) <= 1e-10 * abs(E[1])
    for r in res:
        assert np.abs(r["forces"] - res[1]["forces"]).max() <= 1e-9 * np.abs(res[1]["forces"]).max()
        assert np.abs(r["dEdmu"] - res[1]["dEdmu"]).max() <= 1e-9 * np.abs(res[1]["dEdmu"]).max()
    # and the octupoles matter: without them the energy differs
    e0 = oracle.ewald(pos, q, mu, th, edge=L, eps=1e-14, grad=False)["energy"]
    assert abs(e0 - E[1]) > 1e-3 * abs(E[1])


def test_octupole_translation_invariance():
    import oracle
    pos, q, mu, th, om, L = _octupole_system(6)
    e1 = oracle.ewald(pos, q, mu, th, edge=L, eps=1e-14, omega=om, grad=False)["energy"]
    e2 = oracle.ewald(pos + np.array([1.3, -2.2, 0.7]), q, mu, th, edge=L, eps=1e-14, omega=om,
                      grad=False)["energy"]
    assert abs(e1 - e2) <= 1e-12 * abs(e1)


def test_octupole_is_the_limit_of_a_charge_cube():
    """A point octupole with Omega_xyz = w (and its permutations; traceless) is the limit of eight charges
    s_x s_y s_z 6 w / d^3 at the corners (+-d/2)^3 of a cube around it: the third Taylor term of the
    cluster's potential is d^3 (6w/d^3) d_x d_y d_z = Omega : grad^3.  The cube has no rank-4 moment, and
    its rank-5 moment acts as d_x d_y d_z (Laplacian), which vanishes on the Coulomb potential, so the
    first correction is O(d^4).  The interaction energy with a neutral charge pair, Richardson-
    extrapolated in d^4, matches the oracle's octupole (normalisation Omega : grad grad grad used
    literally, sign, reciprocal factor -i Omega:kkk)."""
    import oracle
    L, w = 14.0, 0.3
    P = np.array([0.4, -0.3, 0.2])
    pair_pos = np.array([[2.9, 1.1, -1.6], [-2.2, 2.4, 1.3]])
    pair_q = np.array([1.0, -1.0])
    om = np.zeros((1, 10))
    om[0, 4] = w          # xyz

    def E(pos, q, omega=None):
        return oracle.ewald(pos, q, edge=L, eps=1e-14, grad=False,
                            mu=np.zeros((len(q), 3)) if omega is not None else None,
                            theta=np.zeros((len(q), 6)) if omega is not None else None, omega=omega)["energy"]

    # interaction of the point octupole with the pair
    e_oct = (E(np.vstack([P, pair_pos]), np.array([0.0, 1.0, -1.0]), np.vstack([om, np.zeros((2, 10))]))
             - E(P[None], np.array([0.0]), om) - E(pair_pos, pair_q))

    def e_cube(d):
        corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
        qc = corners.prod(axis=1) * 6 * w / d ** 3
        pc = P + 0.5 * d * corners
        return E(np.vstack([pc, pair_pos]), np.concatenate([qc, pair_q])) - E(pc, qc) - E(pair_pos, pair_q)

    d = 0.4
    e1, e2 = e_cube(d), e_cube(d / 2)
    rich = (16 * e2 - e1) / 15
    assert abs(e_oct) > 1e-3
    assert abs(e1 - e_oct) <= 1e-4 * abs(e_oct)          # the cube itself: O(d^4)
    assert abs(rich - e_oct) <= 1e-6 * abs(e_oct), (rich, e_oct, e1, e2)


def test_octupole_forces_and_fields_are_derivatives():
    """Central differences of the octupole system's energy in positions and dipoles."""
    import oracle
    pos, q, mu, th, om, L = _octupole_system(7, n=12)
    r = oracle.ewald(pos, q, mu, th, edge=L, eps=1e-14, omega=om)
    h = 1e-5
    for i in (0, 5, 11):
        for c in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, c] += h
            p2[i, c] -= h
            fd = -(oracle.ewald(p1, q, mu, th, edge=L, eps=1e-14, omega=om, grad=False)["energy"]
                   - oracle.ewald(p2, q, mu, th, edge=L, eps=1e-14, omega=om, grad=False)["energy"]) / (2 * h)
            assert fd == pytest.approx(r["forces"][i, c], rel=1e-6, abs=1e-7 * np.abs(r["forces"]).max())
            m1, m2 = mu.copy(), mu.copy()
            m1[i, c] += h
            m2[i, c] -= h
            fd = (oracle.ewald(pos, q, m1, th, edge=L, eps=1e-14, omega=om, grad=False)["energy"]
                  - oracle.ewald(pos, q, m2, th, edge=L, eps=1e-14, omega=om, grad=False)["energy"]) / (2 * h)
            assert fd == pytest.approx(r["dEdmu"][i, c], rel=1e-6, abs=1e-7 * np.abs(r["dEdmu"]).max())

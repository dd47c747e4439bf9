"""Pins of the NumPy transcription of the method (oracle/ankh_ref) against
facts fixed by the mathematics, not by the transcription itself:

* Lagrange property of the Chebyshev basis: S_k(r_j) = delta_kj, and the
  differentiation matrix reproduces T_n' = n U_{n-1};
* anterpolation reproduces polynomial moments exactly (degree < L per axis):
  total charge, dipole moment sum(q x + mu), second moment
  sum(q x x^T + mu x^T + x mu^T + 2 Theta);
* M2M preserves those moments from children to parent;
* the far-image root operator equals a direct image sum of the kernel;
* the 316 M2L operators of a level are those of 16 classes of the cube's
  symmetries with the node indices moved;
* forces and fields are the exact gradient of the approximate energy
  (central finite differences);
* the approximation converges geometrically in L to the classical-Ewald
  value, and agrees across tree depths within the approximation error;
* ANKH-FFT: the reinterpolation onto the equispaced grids preserves the
  polynomial moments it can represent, the transform-based far energy equals
  the plain double sum over leaf pairs and images that defines it, its
  spectrum is real, its leaf local expansions are the gradient of that
  quadratic form, and the method converges to the classical-Ewald value.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import ankh_ref as R


@pytest.mark.parametrize("L", [2, 3, 5, 8])
def test_lagrange_property(L):
    r = R.cheb_nodes(L)
    S = R.cheb_T(r, L) @ R.cheb_H(L).T          # S[j, k] = S_k(r_j)
    np.testing.assert_allclose(S, np.eye(L), atol=1e-13)


@pytest.mark.parametrize("L", [3, 6, 9])
def test_differentiation_matrix(L):
    x = np.linspace(-0.97, 0.97, 11)
    dT = R.cheb_T(x, L) @ R.cheb_D(L).T
    # T_n'(x) = n U_{n-1}(x), U by its own recurrence
    U = np.zeros((len(x), L))
    U[:, 0] = 1
    if L > 1:
        U[:, 1] = 2 * x
    for m in range(2, L):
        U[:, m] = 2 * x * U[:, m - 1] - U[:, m - 2]
    ref = np.zeros_like(dT)
    for n in range(1, L):
        ref[:, n] = n * U[:, n - 1]
    np.testing.assert_allclose(dT, ref, atol=1e-11)
    assert np.allclose(np.triu(R.cheb_D(L)), 0)   # strictly lower triangular


def _leaf_moments(Q, L, centre, h):
    nodes = R.nodes3d(L) * h + centre               # physical node positions
    m0 = Q.sum()
    m1 = nodes.T @ Q
    m2 = np.einsum("ka,kb,k->ab", nodes, nodes, Q)
    return m0, m1, m2


def test_p2m_reproduces_moments():
    rng = np.random.default_rng(1)
    edge, E, L = 10.0, 0, 4
    n = 12
    pos = rng.uniform(-5, 5, (n, 3))
    q = rng.normal(size=n)
    mu = rng.normal(size=(n, 3)) * 0.3
    th = synth.random_traceless_theta(rng, n, 0.2)
    out = R.evaluate(pos, q, mu, th, edge, E, L, 0.1, 2, grad=False, keep=True)
    Q = out["Q"].reshape(-1)
    m0, m1, m2 = _leaf_moments(Q, L, np.zeros(3), 0.5 * edge)
    x = R.wrap(pos, edge)
    Th = np.stack([np.stack([th[:, 0], th[:, 1], th[:, 2]], 1), np.stack([th[:, 1], th[:, 3], th[:, 4]], 1),
                   np.stack([th[:, 2], th[:, 4], th[:, 5]], 1)], 1)
    assert m0 == pytest.approx(q.sum(), abs=1e-12)
    np.testing.assert_allclose(m1, (q[:, None] * x + mu).sum(0), atol=1e-11)
    want = (np.einsum("n,na,nb->ab", q, x, x) + np.einsum("na,nb->ab", mu, x) + np.einsum("na,nb->ab", x, mu)
            + 2 * Th.sum(0))
    np.testing.assert_allclose(m2, want, atol=1e-10)


def test_m2m_preserves_moments():
    rng = np.random.default_rng(2)
    edge, E, L = 12.0, 2, 4
    n = 200
    pos = rng.uniform(-6, 6, (n, 3))
    q = rng.normal(size=n)
    mu = rng.normal(size=(n, 3)) * 0.3
    out = R.evaluate(pos, q, mu, None, edge, E, L, 0.1, 2, grad=False, keep=True)
    M = out["M"]
    for e in range(E):
        ns = 1 << e
        w = edge / ns
        for cell in itertools.product(range(ns), repeat=3):
            c = -0.5 * edge + (np.array(cell) + 0.5) * w
            par = _leaf_moments(M[e][cell], L, c, 0.5 * w)
            acc = [0.0, np.zeros(3), np.zeros((3, 3))]
            for b in itertools.product((0, 1), repeat=3):
                ch = tuple(2 * np.array(cell) + np.array(b))
                cc = -0.5 * edge + (np.array(ch) + 0.5) * (w / 2)
                m = _leaf_moments(M[e + 1][ch], L, cc, 0.25 * w)
                for k in range(3):
                    acc[k] = acc[k] + m[k]
            assert par[0] == pytest.approx(acc[0], abs=1e-11)
            np.testing.assert_allclose(par[1], acc[1], atol=1e-10)
            np.testing.assert_allclose(par[2], acc[2], atol=1e-9)


def test_root_operator_is_image_sum():
    L, edge, xi, p = 3, 7.0, 0.2, 3
    C = R.periodic_root_matrix(edge, L, xi, p)
    g = R.nodes3d(L) * 0.5 * edge
    k, l = 5, 17
    s = 0.0
    for I in itertools.product(range(-p, p + 1), repeat=3):
        if max(map(abs, I)) < 2:
            continue
        r = np.linalg.norm(g[k] - g[l] - edge * np.array(I))
        s += math.erfc(xi * r) / r
    assert C[k, l] == pytest.approx(s, rel=1e-13)
    np.testing.assert_allclose(C, C.T, rtol=1e-13)


@pytest.mark.parametrize("far", ["fmm", "fft"])
def test_reference_gradient_is_exact(far):
    d = synth.water(40, seed=3)
    edge = d["edge"]
    E, L, xi, p = 1, 4, 0.08, 3
    kw = dict(far=far, eq_order=4)
    base = R.evaluate(d["pos"], d["q"], d["mu"], d["theta"], edge, E, L, xi, p, grad=True, **kw)
    h = 1e-5
    for i in (4, 50):
        for c in range(3):
            vals = []
            for s in (1, -1):
                pp = d["pos"].copy()
                pp[i, c] += s * h
                vals.append(R.evaluate(pp, d["q"], d["mu"], d["theta"], edge, E, L, xi, p, grad=False, **kw)["energy"])
            assert -(vals[0] - vals[1]) / (2 * h) == pytest.approx(base["forces"][i, c], rel=1e-6, abs=1e-7)
            vals = []
            for s in (1, -1):
                mm = d["mu"].copy()
                mm[i, c] += s * h
                vals.append(R.evaluate(d["pos"], d["q"], mm, d["theta"], edge, E, L, xi, p, grad=False, **kw)["energy"])
            assert (vals[0] - vals[1]) / (2 * h) == pytest.approx(base["dEdmu"][i, c], rel=1e-6, abs=1e-7)


def test_geometric_convergence_to_ewald():
    d = synth.water(150, seed=8)
    edge = d["edge"]
    ex = oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=edge, eps=1e-13)
    s2 = math.log(10 / 1e-7)
    xi = math.pi / (edge * math.sqrt(s2))
    p = int(math.ceil(math.sqrt(s2) / (xi * edge))) + 1
    errs = []
    for L in (3, 4, 6):
        r = R.evaluate(d["pos"], d["q"], d["mu"], d["theta"], edge, 1, L, xi, p, grad=True)
        errs.append((abs(r["energy"] - ex["energy"]) / abs(ex["energy"]),
                     np.sqrt(np.sum((r["forces"] - ex["forces"]) ** 2) / np.sum(ex["forces"] ** 2))))
    assert errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[0][0] > errs[2][0]
    assert errs[2][0] < 2e-6 and errs[2][1] < 2e-5
    # depth consistency: depth 0 and depth 1 agree within the approximation error
    r0 = R.evaluate(d["pos"], d["q"], d["mu"], d["theta"], edge, 0, 6, xi, p, grad=False)
    assert abs(r0["energy"] - ex["energy"]) < 2e-6 * abs(ex["energy"])


def test_m2l_projector_pins():
    """Compressed M2L: P is the orthogonal projector on the leading singular subspace of the stacked
    operators; full rank reproduces every operator, and the truncation error of the stack equals the
    first dropped singular value (Eckart-Young, spectral norm)."""
    L, w, xi = 4, 6.0, 0.05
    nu = L ** 3
    offs = [d for d in itertools.product(range(-3, 4), repeat=3) if max(abs(c) for c in d) >= 2]
    A = np.hstack([R.m2l_matrix(d, w, L, xi) for d in offs])
    s = np.linalg.svd(A, compute_uv=False)
    P = R.m2l_projector(w, L, xi, nu)
    assert np.max(np.abs(P - np.eye(nu))) < 1e-10
    r = 20
    P = R.m2l_projector(w, L, xi, r)
    assert np.max(np.abs(P @ P - P)) < 1e-12 and np.max(np.abs(P - P.T)) < 1e-14
    err = np.linalg.norm(A - P @ A, 2)
    assert abs(err - s[r]) <= 1e-8 * s[0]
    # K_-d = K_d^T: the projected stack of transposes loses the same
    At = np.hstack([R.m2l_matrix(d, w, L, xi).T for d in offs])
    assert abs(np.linalg.norm(At - P @ At, 2) - s[r]) <= 1e-8 * s[0]


def test_m2l_cube_symmetry_classes():
    """The library evaluates one M2L operator per class of the cube's 48 symmetries and moves the node
    indices for the rest.  Pinned here on the oracle's operators: the 316 far offsets fall into 16
    classes (representatives 3 >= r_x >= r_y >= r_z >= 0, r_x >= 2, each class one orbit of the 48
    axis permutations with reflections); for d = g r, (g v)_c = s_c v_{p_c}, node k maps to k~ with
    k~_{p_c} = k_c (s_c = +1) or L-1-k_c (s_c = -1), and K_d[k, l] = K_r[k~, l~]."""
    L, w, xi = 4, 0.7, 1.3
    offs = R.interaction_offsets()
    reps = sorted({tuple(sorted((abs(c) for c in d), reverse=True)) for d in offs})
    assert len(offs) == 316 and len(reps) == 16
    assert all(r[0] >= 2 and r[0] >= r[1] >= r[2] >= 0 for r in reps)
    group = [(perm, sg) for perm in itertools.permutations(range(3))
             for sg in itertools.product((1, -1), repeat=3)]
    assert len(group) == 48
    for r in reps:   # each class is the orbit of its representative
        orbit = {tuple(sg[c] * r[perm[c]] for c in range(3)) for perm, sg in group}
        assert orbit == {d for d in offs if tuple(sorted((abs(c) for c in d), reverse=True)) == r}
    Kr = {r: R.m2l_matrix(r, w, L, xi) for r in reps}
    idx = np.array(list(itertools.product(range(L), repeat=3)))   # node k -> (k_x, k_y, k_z)
    worst = 0.0
    for d in offs:
        a = [abs(c) for c in d]
        order = sorted(range(3), key=lambda c: -a[c])      # axes by |d_c|, largest first (stable)
        p = [0] * 3
        for j, c in enumerate(order):
            p[c] = j
        r = tuple(a[c] for c in order)
        moved = np.empty_like(idx)
        for c in range(3):
            moved[:, p[c]] = L - 1 - idx[:, c] if d[c] < 0 else idx[:, c]
        kt = (moved[:, 0] * L + moved[:, 1]) * L + moved[:, 2]
        Kd = R.m2l_matrix(d, w, L, xi)
        worst = max(worst, np.max(np.abs(Kd - Kr[r][np.ix_(kt, kt)])) / np.max(np.abs(Kd)))
    assert worst < 1e-14


@pytest.mark.parametrize("L,Le", [(6, 4), (5, 5), (4, 6)])
def test_fft_reinterpolation_preserves_moments(L, Le):
    """The equispaced Lagrange basis reproduces polynomials of degree < Le, so the reinterpolated
    charges keep every moment of that degree: sum_a M_a x_a^m = sum_k Q_k r_k^m."""
    E = R.equi_reinterp(L, Le)
    Q = np.random.default_rng(L * 10 + Le).normal(size=L)
    M = E @ Q
    t, r = R.equi_nodes(Le), R.cheb_nodes(L)
    for m in range(min(Le, L)):
        assert np.sum(M * t ** m) == pytest.approx(np.sum(Q * r ** m), abs=1e-12)
    # Le >= L: the map is exact on the whole Chebyshev space (its own interpolant back is the identity)
    if Le >= L:
        back = R.cheb_T(t, L) @ R.cheb_H(L).T      # S_k(x_a)
        np.testing.assert_allclose(back.T @ E, np.eye(L), atol=1e-12)


@pytest.mark.parametrize("n", [2, 3])
def test_fft_far_equals_its_definition(n):
    """Tiny cell (2 or 3 leaves per axis; ANKH-FFT's single-level grid need not be an octree level):
    the energy through the 6D transform equals the plain sum over leaf pairs, the images of the source
    leaf in the displacement cube and the equispaced nodes; the spectrum of the embedded matrix is
    real; the leaf local expansions are the gradient of the energy in the leaf charges (exact for a
    quadratic form: E(Q+d) - E(Q-d) = 2 d . Lambda)."""
    rng = np.random.default_rng(11)
    edge, E, L, Le, xi, p = 6.0, 1, 3, 3, 0.3, 2
    w = edge / n
    pos = rng.uniform(-3, 3, (10, 3))
    q = rng.normal(size=10)
    mu = 0.3 * rng.normal(size=(10, 3))
    th = synth.random_traceless_theta(rng, 10, 0.2)
    Q = R.evaluate(pos, q, mu, th, edge, E, L, xi, p, grad=False, keep=True, far="fft", eq_order=Le,
                   leaves=n)["Q"].reshape(n ** 3, L ** 3)
    K = R.fft_kernel_table(n, w, Le, xi, p)
    e, Lam, D = R.fft_far(Q, n, L, Le, K)
    dense = R.fft_far_dense(Q, n, w, L, Le, xi, p)
    assert e == pytest.approx(dense, rel=1e-12)
    assert np.max(np.abs(D.imag)) <= 1e-12 * np.max(np.abs(D.real))
    assert 0.5 * np.sum(Q * Lam) == pytest.approx(e, rel=1e-12)
    d = rng.normal(size=Q.shape)
    ep, em = R.fft_far(Q + d, n, L, Le, K)[0], R.fft_far(Q - d, n, L, Le, K)[0]
    assert (ep - em) / 2 == pytest.approx(np.sum(d * Lam), rel=1e-10)


def test_fft_far_field_converges_to_ewald():
    """ANKH-FFT converges in the equispaced order to the classical-Ewald value and, at the order of
    the Chebyshev grids, matches the accuracy of the multilevel far field."""
    d = synth.water(150, seed=8)
    edge = d["edge"]
    ex = oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=edge, eps=1e-13)
    s2 = math.log(10 / 1e-7)
    xi = math.pi / (edge * math.sqrt(s2))
    p = int(math.ceil(math.sqrt(s2) / (xi * edge))) + 1
    errs = []
    for Le in (3, 4, 6):
        r = R.evaluate(d["pos"], d["q"], d["mu"], d["theta"], edge, 1, 6, xi, p, grad=True, far="fft", eq_order=Le)
        errs.append((abs(r["energy"] - ex["energy"]) / abs(ex["energy"]),
                     np.sqrt(np.sum((r["forces"] - ex["forces"]) ** 2) / np.sum(ex["forces"] ** 2))))
        assert r["e_per"] == 0.0
    assert errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[0][0] > errs[2][0]
    assert errs[2][0] < 2e-6 and errs[2][1] < 2e-5
    # a leaf grid that is not an octree level (3 per axis) reaches the same accuracy
    r3 = R.evaluate(d["pos"], d["q"], d["mu"], d["theta"], edge, 1, 6, xi, p, grad=True, far="fft", eq_order=6,
                    leaves=3)
    assert abs(r3["energy"] - ex["energy"]) < 2e-6 * abs(ex["energy"])
    assert np.sqrt(np.sum((r3["forces"] - ex["forces"]) ** 2) / np.sum(ex["forces"] ** 2)) < 2e-5


# ---- octupoles -------------------------------------------------------------------------------------------

def test_p2m_reproduces_octupole_moment():
    """Interpolation of order L >= 4 reproduces cubic polynomials, so the third moment of the leaf's modified
    charges is sum (q x_a x_b x_c + mu-, Theta- terms + 6 Omega_abc): the octupole enters P2M through
    Omega : grad^3 with the right normalisation."""
    rng = np.random.default_rng(11)
    edge, E, L = 10.0, 0, 5
    n = 10
    pos = rng.uniform(-5, 5, (n, 3))
    q = np.zeros(n)
    om = synth.random_traceless_omega(rng, n, 0.3)
    out = R.evaluate(pos, q, np.zeros((n, 3)), np.zeros((n, 6)), edge, E, L, 0.1, 2, grad=False, keep=True,
                     omega=om)
    Q = out["Q"].reshape(-1)
    nodes = R.nodes3d(L) * 0.5 * edge
    m3 = np.einsum("ka,kb,kc,k->abc", nodes, nodes, nodes, Q)
    full = np.zeros((n, 3, 3, 3))
    for c, (a, b, cc) in enumerate(R.OMEGA_ABC):
        idx = [0] * a + [1] * b + [2] * cc
        for perm in set(itertools.permutations(idx)):
            full[:, perm[0], perm[1], perm[2]] = om[:, c]
    np.testing.assert_allclose(m3, 6 * full.sum(0), atol=1e-10)
    # no lower moments from pure octupoles
    assert abs(Q.sum()) < 1e-11


@pytest.mark.parametrize("far", ["fmm", "fft"])
def test_octupole_gradient_is_exact(far):
    """With octupoles, forces and fields of the transcription are central differences of its own energy
    (P2M with the third derivatives of the basis, L2P with the fourth)."""
    d = synth.water(30, seed=4)
    om = synth.water_octupoles(30, seed=4)
    edge = d["edge"]
    E, L, xi, p = 1, 4, 0.08, 3
    kw = dict(far=far, eq_order=4, omega=om)
    base = R.evaluate(d["pos"], d["q"], d["mu"], d["theta"], edge, E, L, xi, p, grad=True, **kw)
    h = 1e-5
    for i in (3, 41):
        for c in range(3):
            vals = []
            for s in (1, -1):
                pp = d["pos"].copy()
                pp[i, c] += s * h
                vals.append(R.evaluate(pp, d["q"], d["mu"], d["theta"], edge, E, L, xi, p, grad=False, **kw)["energy"])
            assert -(vals[0] - vals[1]) / (2 * h) == pytest.approx(base["forces"][i, c], rel=1e-6, abs=1e-7)
            vals = []
            for s in (1, -1):
                mm = d["mu"].copy()
                mm[i, c] += s * h
                vals.append(R.evaluate(d["pos"], d["q"], mm, d["theta"], edge, E, L, xi, p, grad=False, **kw)["energy"])
            assert (vals[0] - vals[1]) / (2 * h) == pytest.approx(base["dEdmu"][i, c], rel=1e-6, abs=1e-7)


def test_octupole_convergence_to_ewald():
    """With octupoles on every atom, the interpolated energy and forces approach the classical-Ewald oracle
    as the order grows."""
    d = synth.water(100, seed=9)
    om = synth.water_octupoles(100, seed=9)
    edge = d["edge"]
    ex = oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=edge, eps=1e-13, omega=om)
    s2 = math.log(10 / 1e-7)
    xi = math.pi / (edge * math.sqrt(s2))
    p = int(math.ceil(math.sqrt(s2) / (xi * edge))) + 1
    errs = []
    for L in (4, 6, 8):
        r = R.evaluate(d["pos"], d["q"], d["mu"], d["theta"], edge, 1, L, xi, p, grad=True, omega=om)
        errs.append((abs(r["energy"] - ex["energy"]) / abs(ex["energy"]),
                     np.sqrt(np.sum((r["forces"] - ex["forces"]) ** 2) / np.sum(ex["forces"] ** 2))))
    assert errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[2][0] < 1e-6 and errs[2][1] < 1e-5, errs

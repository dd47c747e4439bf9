"""Pins of the induced-dipole oracle (oracle/polarize.py), on the CPU.

* Closed forms of two polarisable atoms (mutual induction along the axis, and
  the transverse field of a fixed dipole), in a box large enough that the
  periodic images change the result by < 2e-5 relative (tin-foil images of a
  pair r apart in a box of edge L act as a field of order 4 pi r^3 / (3 L^3)
  of the direct one).
* Conjugate gradients against the dense solve of the same system.
* The solution minimises the polarisation energy evaluated through the
  oracle's ENERGY (not its fields): U(mu + t d) - U(mu) is quadratic in t with
  no linear term.
"""
import numpy as np
import pytest

import synth
from oracle import polarize as P

L_BIG = 200.0


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def test_two_body_axial_mutual_induction():
    # +q at A and -q at B on the z axis: both feel q / r^2 along +z; each induced dipole adds
    # 2 mu / r^3 on the axis at the other atom.  mu_A = a_A (E + 2 mu_B / r^3) and the same for B.
    r, q, aA, aB = 2.0, 0.8, 0.9, 0.6
    pos = np.array([[0.0, 0.0, -r / 2], [0.0, 0.0, r / 2]])
    mu_ind = P.induce_direct(pos, np.array([q, -q]), None, None, [aA, aB], L_BIG)
    E = q / r ** 2
    den = 1.0 - 4.0 * aA * aB / r ** 6
    want = np.array([aA * E * (1 + 2 * aB / r ** 3) / den, aB * E * (1 + 2 * aA / r ** 3) / den])
    assert np.max(np.abs(mu_ind[:, :2])) <= 1e-9
    np.testing.assert_allclose(mu_ind[:, 2], want, rtol=1e-4)
    # and the induction is a real correction (the mutual term is > 10 % here)
    assert abs(want[0] / (aA * E) - 1) > 0.1


def test_transverse_field_of_a_fixed_dipole():
    # a non-polarisable dipole p x at the origin, a polarisable neutral atom at r z:
    # the field there is -p x / r^3, so mu_ind = -alpha p / r^3 x, and the fixed atom gets nothing
    r, p, a = 2.5, 0.7, 0.4
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    mu = np.array([[p, 0.0, 0.0], [0.0, 0.0, 0.0]])
    mu_ind = P.induce_direct(pos, np.zeros(2), mu, None, [0.0, a], L_BIG)
    assert np.all(mu_ind[0] == 0.0)
    np.testing.assert_allclose(mu_ind[1], [-a * p / r ** 3, 0.0, 0.0], rtol=1e-4, atol=1e-9)


def _tiny_water():
    d = synth.water(4, seed=11)
    return d, synth.water_polarisabilities(4)


def test_cg_matches_dense_solve():
    d, alpha = _tiny_water()
    direct = P.induce_direct(d["pos"], d["q"], d["mu"], d["theta"], alpha, d["edge"], eps=1e-12)
    cg, it, res = P.induce_cg(d["pos"], d["q"], d["mu"], d["theta"], alpha, d["edge"], eps=1e-12, tol=1e-12)
    assert res <= 1e-12 and 0 < it <= 36
    assert rel_rms(cg, direct) <= 1e-10


def test_solution_minimises_the_polarisation_energy():
    d, alpha = _tiny_water()
    args = (d["pos"], d["q"], d["mu"], d["theta"], alpha)
    mu_ind = P.induce_direct(*args, d["edge"], eps=1e-12)
    U0 = P.polarisation_energy(*args, mu_ind, d["edge"])
    delta = np.random.default_rng(5).normal(0.0, 1e-3, mu_ind.shape)
    dU = {t: P.polarisation_energy(*args, mu_ind + t * delta, d["edge"]) - U0 for t in (-1.0, 1.0, 2.0)}
    assert dU[1.0] > 0.0
    assert abs(dU[2.0] / dU[1.0] - 4.0) <= 1e-6               # quadratic in t
    assert abs(dU[1.0] - dU[-1.0]) <= 1e-6 * dU[1.0]          # no linear term: a stationary point


def test_zero_polarisability_and_no_field():
    d, alpha = _tiny_water()
    mu_ind, it, res = P.induce_cg(d["pos"], d["q"], d["mu"], d["theta"], np.zeros_like(alpha), d["edge"])
    assert it == 0 and np.all(mu_ind == 0.0)
    n = len(d["q"])
    mu_ind, it, res = P.induce_cg(d["pos"], np.zeros(n), None, None, alpha, d["edge"])
    assert it == 0 and np.all(mu_ind == 0.0)


def test_rejects_negative_polarisability():
    d, alpha = _tiny_water()
    alpha[3] = -0.1
    with pytest.raises(ValueError):
        P.induce_cg(d["pos"], d["q"], d["mu"], d["theta"], alpha, d["edge"])

"""GPU parity of the induced-dipole solve (ankh_induce, through the C ABI).

* Against the oracle (conjugate gradients on classical Ewald, pinned in
  test_polarize_pins.py): induced dipoles, the polarisation energy U and the
  forces at the solution, within the approximation's tolerance (the bar of the
  other oracle comparisons: 1e-6 relative energy, 1e-5 relative RMS vectors).
* Properties at the benchmark's size (288,000 atoms): the solution satisfies
  its own stationarity condition (one more evaluation), the mixed modes agree
  with FP64, a solve is bitwise reproducible.
* Forces are the gradient of U (central differences of the GPU's own U,
  re-solved at each displaced position).
* Edge cases: no polarisable atom, no field, a negative polarisability, bad
  arguments, the iteration cap.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import polarize as P  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ak():
    import paper_2212_08284_amd as ak
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ak.load_library()
    return ak


def T(a):
    return None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda:0")


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def _water(n_mol, seed):
    d = synth.water(n_mol, seed=seed)
    return d, synth.water_polarisabilities(n_mol)


def _solve(ak, d, alpha, eps=1e-8, prec="fp64", tol=1e-10, forces=True, **ov):
    pl = ak.Plan(len(d["q"]), 0.5 * d["edge"], eps, 2, prec, **ov)
    mi, e, F, it, res = pl.induce(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(alpha), tol=tol,
                                  max_iter=200, forces=forces)
    return pl, mi.cpu().numpy(), e.item(), None if F is None else F.cpu().numpy(), it, res


@pytest.mark.parametrize("far", ["fmm", "fft"])
def test_induce_vs_oracle(ak, far):
    d, alpha = _water(300, 7)
    pl, mi, U, F, it, res = _solve(ak, d, alpha, far=far)
    assert res <= 1e-10 and 0 < it < 60
    ref, it_ref, res_ref = P.induce_cg(d["pos"], d["q"], d["mu"], d["theta"], alpha, d["edge"], eps=1e-11,
                                       tol=1e-11)
    assert rel_rms(mi, ref) <= 1e-5
    U_ref = P.polarisation_energy(d["pos"], d["q"], d["mu"], d["theta"], alpha, ref, d["edge"])
    assert abs(U - U_ref) <= 1e-6 * abs(U_ref)
    # forces at the solution: the Ewald forces of the total dipoles
    F_ref = oracle.ewald(d["pos"], d["q"], d["mu"] + ref, d["theta"], edge=d["edge"], eps=1e-11)["forces"]
    assert rel_rms(F, F_ref) <= 1e-5
    pl.close()


def test_induce_without_permanent_dipoles_or_quadrupoles(ak):
    d, alpha = _water(300, 9)
    pl = ak.Plan(len(d["q"]), 0.5 * d["edge"], 1e-8, 1, "fp64")
    mi, e, F, it, res = pl.induce(T(d["pos"]), T(d["q"]), None, None, T(alpha), tol=1e-10)
    ref, _, _ = P.induce_cg(d["pos"], d["q"], None, None, alpha, d["edge"], eps=1e-11, tol=1e-11)
    assert rel_rms(mi.cpu().numpy(), ref) <= 1e-5
    U_ref = P.polarisation_energy(d["pos"], d["q"], None, None, alpha, ref, d["edge"])
    assert abs(e.item() - U_ref) <= 1e-6 * abs(U_ref)
    pl.close()


def _away_from_faces(pos, edge, depth, h, count, seed):
    w = edge / (1 << depth)
    x = pos + 0.5 * edge
    frac = (x / w) - np.floor(x / w)
    ok = np.all((frac * w > 20 * h) & ((1 - frac) * w > 20 * h), axis=1)
    return np.random.default_rng(seed).choice(np.nonzero(ok)[0], count, replace=False)


def test_forces_are_the_gradient_of_the_polarisation_energy(ak):
    d, alpha = _water(300, 13)
    n = len(d["q"])
    pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64")
    args = lambda p: (T(p), T(d["q"]), T(d["mu"]), T(d["theta"]), T(alpha))
    mi, e, F, it, res = pl.induce(*args(d["pos"]), tol=1e-13, max_iter=300, forces=True)
    F = F.cpu().numpy()
    h = 1e-5
    for i in _away_from_faces(d["pos"], d["edge"], pl.stats["depth"], h, 3, 1):
        for c in range(3):
            pp, pm = d["pos"].copy(), d["pos"].copy()
            pp[i, c] += h
            pm[i, c] -= h
            Up = pl.induce(*args(pp), tol=1e-13, max_iter=300)[1].item()
            Um = pl.induce(*args(pm), tol=1e-13, max_iter=300)[1].item()
            fd = -(Up - Um) / (2 * h)
            assert fd == pytest.approx(F[i, c], rel=1e-6, abs=1e-6 * np.abs(F).max()), (i, c)
    pl.close()


def test_induce_water_288000_properties(ak):
    # the benchmark's box: stationarity of the solution, mixed vs FP64, reproducibility
    d = synth.workload("water_288000")
    n = len(d["q"])
    alpha = synth.water_polarisabilities(n // 3)
    tol = 1e-7
    sols = {}
    for prec in ("fp64", "mixed_bf16x3"):
        pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, prec)
        mi, e, F, it, res = pl.induce(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(alpha), tol=tol)
        assert res <= tol and it < 60
        # stationarity: dE/dmu at mu + mu_ind plus mu_ind / alpha vanishes, scaled by sqrt(alpha) as in
        # the solver, relative to the scaled right-hand side
        _, _, g = pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]) + mi, T(d["theta"]))
        _, _, g0 = pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
        s = np.sqrt(alpha)[:, None]
        m = mi.cpu().numpy()
        r = s * g.cpu().numpy() + m / s
        b = s * g0.cpu().numpy()
        assert np.linalg.norm(r) <= (10 * tol if prec == "fp64" else 1e-5) * np.linalg.norm(b)
        if prec == "fp64":
            mi2 = pl.induce(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(alpha), tol=tol)[0]
            assert torch.equal(mi, mi2)
        sols[prec] = m
        pl.close()
    assert rel_rms(sols["mixed_bf16x3"], sols["fp64"]) <= 1e-5


def test_induce_edge_cases(ak):
    d, alpha = _water(50, 3)
    n = len(d["q"])
    pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64")
    a = (T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    # nothing polarisable: zero induced dipoles, U = E, no product
    mi, e, F, it, res = pl.induce(*a, T(np.zeros(n)), forces=True)
    e0, F0, _ = pl.energy_forces(*a)
    assert it == 0 and res == 0.0 and float(mi.abs().max()) == 0.0
    assert e.item() == e0.item() and torch.equal(F, F0)
    # no field: no charges, dipoles or quadrupoles
    mi, e, F, it, res = pl.induce(T(d["pos"]), T(np.zeros(n)), None, None, T(alpha))
    assert it == 0 and float(mi.abs().max()) == 0.0 and e.item() == 0.0
    # a negative polarisability is latched and reported by the sync inside induce
    bad = alpha.copy()
    bad[5] = -1.0
    with pytest.raises(ak.AnkhError) as ei:
        pl.induce(*a, T(bad))
    assert ei.value.status == 1
    # host-checked arguments
    for kw in (dict(tol=0.0), dict(tol=float("nan")), dict(max_iter=-1)):
        with pytest.raises(ak.AnkhError) as ei:
            pl.induce(*a, T(alpha), **kw)
        assert ei.value.status == 1
    # the iteration cap: not converged, the last iterate is still written
    with pytest.raises(ak.AnkhError) as ei:
        pl.induce(*a, T(alpha), tol=1e-14, max_iter=2)
    assert ei.value.status == 8
    mi, e, F, it, res = pl.induce(*a, T(alpha), tol=1e-14, max_iter=2, check=False)
    assert it == 2 and 0 < res < 1 and float(mi.abs().max()) > 0
    # a charges-only plan cannot hold dipoles
    pq = ak.Plan(n, 0.5 * d["edge"], 1e-6, 0, "fp64")
    with pytest.raises(ak.AnkhError):
        pq.induce(T(d["pos"]), T(d["q"]), None, None, T(alpha))
    pq.close()
    pl.close()

"""GPU parity of the charge and quadrupole derivatives (ankh_energy_derivs, through the C ABI).

* Against the oracle (classical Ewald, pinned in test_oracle_pins.py: the
  rock-salt site potential, a point charge's field gradient, central
  differences): dE/dq and the traceless dE/dTheta within the approximation's
  tolerance (1e-5 relative RMS, the bar of the other oracle comparisons).
* They are the exact derivatives of the approximate energy: central
  differences of the GPU's own energy in q_i and along traceless Theta_i
  directions (positions fixed, so no leaf boundary is crossed).
* The mixed modes against FP64; the energy, forces and fields of the same
  call equal those of ankh_energy_forces; optional outputs and errors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

TRACELESS = [np.array(v, dtype=np.float64) for v in
             ([0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0], [0, 0, 0, 0, 1, 0], [1, 0, 0, -1, 0, 0], [1, 0, 0, 0, 0, -1])]


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


def _derivs(pl, d, **kw):
    out = pl.energy_derivs(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), **kw)
    pl.sync()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_derivs_vs_oracle(ak):
    d = synth.water(300, seed=7)
    pl = ak.Plan(len(d["q"]), 0.5 * d["edge"], 1e-8, 2, "fp64")
    o = _derivs(pl, d)
    ref = oracle.ewald_moments(d["pos"], d["q"], d["mu"], d["theta"], edge=d["edge"], eps=1e-11)
    assert rel_rms(o["dEdq"], ref["dEdq"]) <= 1e-5
    assert rel_rms(o["dEdtheta"], ref["dEdtheta"]) <= 1e-5
    # the reported quadrupole derivative is traceless
    assert np.max(np.abs(o["dEdtheta"][:, 0] + o["dEdtheta"][:, 3] + o["dEdtheta"][:, 5])) <= \
        1e-12 * np.max(np.abs(o["dEdtheta"]))
    # the energy, forces and fields of the same call are those of ankh_energy_forces
    e, F, G = pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    assert o["energy"][0] == e.item()
    assert np.array_equal(o["forces"], F.cpu().numpy()) and np.array_equal(o["dEdmu"], G.cpu().numpy())
    pl.close()


def test_derivs_are_gradients_of_the_energy(ak):
    d = synth.water(300, seed=23)
    n = len(d["q"])
    pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64")
    o = _derivs(pl, d, forces=False, fields=False)
    E = lambda q_, th_: pl.energy(T(d["pos"]), T(q_), T(d["mu"]), T(th_)).item()
    h = 1e-5
    scale_q = np.abs(o["dEdq"]).max()
    scale_t = np.abs(o["dEdtheta"]).max()
    for i in np.random.default_rng(2).choice(n, 4, replace=False):
        q1, q2 = d["q"].copy(), d["q"].copy()
        q1[i] += h
        q2[i] -= h
        fd = (E(q1, d["theta"]) - E(q2, d["theta"])) / (2 * h)
        assert fd == pytest.approx(o["dEdq"][i], rel=1e-6, abs=1e-6 * scale_q), i
        for dl in TRACELESS:
            t1, t2 = d["theta"].copy(), d["theta"].copy()
            t1[i] += h * dl
            t2[i] -= h * dl
            fd = (E(d["q"], t1) - E(d["q"], t2)) / (2 * h)
            assert fd == pytest.approx(o["dEdtheta"][i] @ dl, rel=1e-6, abs=1e-6 * scale_t), (i, dl)
    pl.close()


@pytest.mark.parametrize("mode", ["mixed", "mixed_bf16x3"])
def test_derivs_mixed_vs_fp64(ak, mode):
    d = synth.workload("water_9000")
    n = len(d["q"])
    out = {}
    for prec in ("fp64", mode):
        pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, prec)
        out[prec] = _derivs(pl, d, forces=False, fields=False)
        pl.close()
    assert rel_rms(out[mode]["dEdq"], out["fp64"]["dEdq"]) <= 1e-4
    assert rel_rms(out[mode]["dEdtheta"], out["fp64"]["dEdtheta"]) <= 1e-4


def test_derivs_optional_outputs_and_errors(ak):
    d = synth.water(100, seed=4)
    n = len(d["q"])
    pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64")
    full = _derivs(pl, d)
    only_q = _derivs(pl, d, forces=False, fields=False, theta_grad=False)
    assert set(only_q) == {"energy", "dEdq"}
    assert np.array_equal(only_q["dEdq"], full["dEdq"]) and only_q["energy"][0] == full["energy"][0]
    only_t = _derivs(pl, d, forces=False, fields=False, potentials=False)
    assert np.array_equal(only_t["dEdtheta"], full["dEdtheta"])
    # without quadrupoles the derivative in Theta is still defined (at Theta = 0)
    nq = pl.energy_derivs(T(d["pos"]), T(d["q"]), T(d["mu"]), None)
    ref = oracle.ewald_moments(d["pos"], d["q"], d["mu"], None, edge=d["edge"], eps=1e-11)
    assert rel_rms(nq["dEdtheta"].cpu().numpy(), ref["dEdtheta"]) <= 1e-4
    assert rel_rms(nq["dEdq"].cpu().numpy(), ref["dEdq"]) <= 1e-4
    pl.close()
    # a plan without quadrupoles cannot give dE/dTheta; charges-only plans give potentials
    p1 = ak.Plan(n, 0.5 * d["edge"], 1e-6, 1, "fp64")
    with pytest.raises(ak.AnkhError) as ei:
        p1.energy_derivs(T(d["pos"]), T(d["q"]), T(d["mu"]), None)
    assert ei.value.status == 1
    p0 = ak.Plan(n, 0.5 * d["edge"], 1e-6, 0, "fp64")
    o0 = p0.energy_derivs(T(d["pos"]), T(d["q"]), None, None, forces=True, fields=False, theta_grad=False)
    ref0 = oracle.ewald_moments(d["pos"], d["q"], None, None, edge=d["edge"], eps=1e-11)
    assert rel_rms(o0["dEdq"].cpu().numpy(), ref0["dEdq"]) <= 1e-4
    p1.close()
    p0.close()

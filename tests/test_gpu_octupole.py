"""GPU parity of the octupole path (ankh_energy_octupole: the operator of eq. 1 extended by
Omega : grad^3, the next multipole order that the paper's introduction names).

* Stage parity against the NumPy transcription (oracle/ankh_ref with omega): the same approximation,
  so energy terms, leaf modified charges, forces and fields agree to rounding in FP64, on both far
  fields, at depths whose leaves hold more than one P2M chunk and more than one pair-kernel chunk
  (gather form), one chunk (own-leaf round robin) and none (empty leaves), and on the three forms of
  the near-field erfc.
* Method parity against the classical-Ewald oracle with octupoles (oracle.ewald(omega=...)).
* The mixed path against the FP64 path; energy-only and fields-only calls; octupoles of zero against
  the quadrupole path; a latched trace error; host-checked argument errors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import ankh_ref  # noqa: E402

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


def _water(n_mol=300, seed=7):
    d = synth.water(n_mol, seed=seed)
    d["omega"] = synth.water_octupoles(n_mol, seed=seed)
    return d


def _run(ak, d, eps=1e-6, prec="fp64", forces=True, fields=True, **ov):
    pl = ak.Plan(len(d["q"]), 0.5 * d["edge"], eps, 3, prec, **ov)
    e, F, G = pl.energy_octupole(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(d["omega"]),
                                 forces=forces, fields=fields)
    pl.sync()
    return (pl, e.item(), None if F is None else F.cpu().numpy(), None if G is None else G.cpu().numpy())


def _check_terms(pl, e, F, G, r, far):
    terms = pl.last_terms()
    scale = abs(r["e_near"]) + abs(r["e_self"]) + 1.0
    assert abs(terms["near"] - r["e_near"]) <= 1e-12 * scale
    assert abs(terms["far_levels"] - sum(r["e_far_levels"])) <= 1e-12 * scale
    if far == "fmm":
        assert abs(terms["periodic"] - r["e_per"]) <= 1e-12 * scale
    assert abs(terms["self"] - r["e_self"]) <= 1e-12 * scale
    assert abs(e - r["energy"]) <= 1e-12 * scale
    assert rel_rms(F, r["forces"]) <= 1e-11
    assert rel_rms(G, r["dEdmu"]) <= 1e-11


@pytest.mark.parametrize("depth,order", [(0, 4), (1, 5), (2, 5), (3, 4), (4, 4)])
def test_octupole_stage_parity_fmm(ak, depth, order):
    """Depth 0 and 1: leaves of 900 and ~110 atoms (several P2M chunks of 32, the pair kernel's gather form);
    depth 2: ~14 atoms (own-leaf round robin); depths 3 and 4: the two short-series forms of erfc."""
    d = _water()
    pl, e, F, G = _run(ak, d, far="fmm", depth=depth, order=order, images=4, m2l_tol=-1.0)
    st = pl.stats
    assert st["max_order"] == 3 and st["depth"] == depth and st["order"] == order
    r = ankh_ref.evaluate(d["pos"], d["q"], d["mu"], d["theta"], d["edge"], st["depth"], st["order"], st["xi"],
                          st["images"], grad=True, keep=True, root_order=st["root_order"], omega=d["omega"])
    Q = pl.leaf_multipoles()
    Qr = r["Q"].reshape(Q.shape)
    assert np.max(np.abs(Q - Qr)) <= 1e-12 * np.max(np.abs(Qr))
    _check_terms(pl, e, F, G, r, "fmm")
    pl.close()


@pytest.mark.parametrize("kw", [dict(depth=2, order=5, eq_order=5), dict(leaves=12, order=4, eq_order=4),
                                dict(leaves=3, order=6, eq_order=6)])
def test_octupole_stage_parity_fft(ak, kw):
    """ANKH-FFT: an octree level, a 12^3 grid with empty leaves, and a 3^3 grid (direct DFTs)."""
    d = _water()
    pl, e, F, G = _run(ak, d, far="fft", images=3, **kw)
    st = pl.stats
    assert st["far_field"] == ak.ANKH_FAR_FFT
    leaves = kw.get("leaves")
    r = ankh_ref.evaluate(d["pos"], d["q"], d["mu"], d["theta"], d["edge"], max(st["depth"], 0), st["order"],
                          st["xi"], st["images"], grad=True, far="fft", eq_order=kw["eq_order"], leaves=leaves,
                          omega=d["omega"])
    _check_terms(pl, e, F, G, r, "fft")
    pl.close()


@pytest.fixture(scope="module")
def ewald_600():
    d = _water(200)
    return d, oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=d["edge"], eps=1e-12, omega=d["omega"])


@pytest.mark.parametrize("far,eps,etol,ftol", [("fmm", 1e-8, 1e-7, 1e-6), ("fft", 1e-6, 1e-6, 1e-5)])
def test_octupole_vs_oracle(ak, ewald_600, far, eps, etol, ftol):
    """The planned evaluation against classical Ewald with the same octupoles (the oracle's real and
    reciprocal sums carry Omega : grad^3 and -i Omega : kkk)."""
    d, ref = ewald_600
    pl, e, F, G = _run(ak, d, eps=eps, far=far)
    rel_e = abs(e - ref["energy"]) / abs(ref["energy"])
    rf, rg = rel_rms(F, ref["forces"]), rel_rms(G, ref["dEdmu"])
    print(f"octupoles {far} eps={eps}: order {pl.stats['order']} rel_E={rel_e:.2e} rel_F={rf:.2e} rel_G={rg:.2e}")
    assert rel_e < etol and rf < ftol and rg < ftol
    pl.close()


@pytest.mark.parametrize("prec,far", [("mixed", "fft"), ("mixed", "fmm"), ("mixed_bf16x3", "fmm")])
def test_octupole_mixed_vs_fp64(ak, prec, far):
    d = _water()
    _, e0, F0, G0 = _run(ak, d, far=far)
    pl, e1, F1, G1 = _run(ak, d, prec=prec, far=far)
    assert pl.stats["near_precision"] == 1
    assert abs(e1 - e0) < 1e-5 * abs(e0)
    assert rel_rms(F1, F0) < 1e-4 and rel_rms(G1, G0) < 1e-4
    pl.close()


def test_octupole_energy_only_and_fields_only(ak):
    d = _water()
    pl, e, F, G = _run(ak, d, far="fmm", depth=2, order=5)
    e1 = pl.energy_octupole(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(d["omega"]), forces=False,
                            fields=False)[0].item()
    _, _, G2 = pl.energy_octupole(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(d["omega"]), forces=False,
                                  fields=True)
    pl.sync()
    assert abs(e1 - e) <= 1e-13 * abs(e)
    assert rel_rms(G2.cpu().numpy(), G) <= 1e-14
    pl.close()


def test_octupole_zero_matches_quadrupole_path(ak):
    """Omega = 0 through the octupole kernels gives the quadrupole path's result (up to rounding), and a
    plan for octupoles serves the lower-order calls."""
    d = _water()
    d["omega"] = np.zeros_like(d["omega"])
    pl, e, F, G = _run(ak, d, far="fft")
    e2, F2, G2 = pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    pl.sync()
    assert abs(e2.item() - e) <= 1e-13 * abs(e)
    assert rel_rms(F2.cpu().numpy(), F) <= 1e-13 and rel_rms(G2.cpu().numpy(), G) <= 1e-13
    pl.close()


def test_octupole_bitwise_reproducible(ak):
    d = _water()
    pl, e, F, G = _run(ak, d, far="fft")
    e2, F2, G2 = pl.energy_octupole(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(d["omega"]))
    pl.sync()
    assert e2.item() == e and np.array_equal(F2.cpu().numpy(), F) and np.array_equal(G2.cpu().numpy(), G)
    pl.close()


def test_octupole_with_charges_only(ak):
    """Charges and octupoles without dipoles or quadrupoles (mu, theta NULL): the gather fills zero
    moments, and the field dE/dmu is the one at mu = 0."""
    d = _water()
    n = len(d["q"])
    pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 3, "fp64", far="fmm", depth=2, order=5, images=4, m2l_tol=-1.0)
    e, F, G = pl.energy_octupole(T(d["pos"]), T(d["q"]), None, None, T(d["omega"]))
    pl.sync()
    st = pl.stats
    r = ankh_ref.evaluate(d["pos"], d["q"], np.zeros((n, 3)), None, d["edge"], st["depth"], st["order"], st["xi"],
                          st["images"], grad=True, root_order=st["root_order"], omega=d["omega"])
    scale = abs(r["e_near"]) + abs(r["e_self"]) + 1.0
    assert abs(e.item() - r["energy"]) <= 1e-12 * scale
    assert rel_rms(F.cpu().numpy(), r["forces"]) <= 1e-11
    assert rel_rms(G.cpu().numpy(), r["dEdmu"]) <= 1e-11
    pl.close()


def test_octupole_errors(ak):
    d = _water(100)
    n = len(d["q"])
    # a trace Omega_aab that does not vanish is latched and reported by sync
    om = d["omega"].copy()
    om[5, 0] += 0.01                     # xxx: trace Omega_aax
    pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 3, "fp64")
    pl.energy_octupole(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(om))
    with pytest.raises(ak.AnkhError) as ex:
        pl.sync()
    assert ex.value.status == 3
    pl.sync()                            # cleared
    # non-finite octupoles
    om = d["omega"].copy()
    om[7, 4] = np.nan
    pl.energy_octupole(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(om))
    with pytest.raises(ak.AnkhError) as ex:
        pl.sync()
    assert ex.value.status == 2
    pl.close()
    # a plan without octupoles refuses them (host check, nothing enqueued)
    pl2 = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64")
    with pytest.raises(ak.AnkhError) as ex:
        pl2.energy_octupole(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]), T(d["omega"]))
    assert ex.value.status == 1
    pl2.close()

"""GPU parity of the ANKH-FFT far field (far="fft", through the C ABI).

* Stage parity against the NumPy transcription (oracle/ankh_ref, far="fft"):
  same depth, orders, xi and images, so the far energy, the total, forces and
  fields agree to rounding (FP64), at depths 0-3, equispaced orders below,
  equal to and above the Chebyshev order, charges only / +dipoles /
  +quadrupoles.
* Method parity against the classical-Ewald oracle (the stored water_9000
  values): FP64 within 1e-6 relative energy and 1e-5 relative RMS force and
  field, like ANKH-FMM.
* The forces and fields are the exact gradient of the approximate energy
  (central differences of the GPU FP64 energy).
* Full size (288,000-atom water box, depth 4, the benchmark's sizes): the
  mixed modes against FP64, and FP64 against the ANKH-FMM path (both
  approximate the same energy within the accuracy target) and against the
  oracle on the stored sampled atoms.
* Depths 5 and 6 (the cell transforms in three passes through HBM; the same
  passes are forced at small depths for the stage parity): against ANKH-FMM
  at the same depth on the 288,000- and 9,000,000-atom boxes.
* Leaf grids that are not octree levels (any count per axis up to 40): stage
  parity, finite differences, and the benchmark box on 20^3 leaves.
* Planning errors: depth beyond 6, equispaced order out of range.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import ankh_ref  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _system(kind, seed=7):
    if kind == "qmt":
        return synth.water(300, seed=seed)
    if kind == "qm":
        return synth.water(300, seed=seed, with_theta=False)
    if kind == "q":
        d = synth.charges(700, 17.0, seed=seed)
        d["q"][0] += 0.25                      # non-neutral: background term
        return d
    raise KeyError(kind)


def _run(ak, d, eps=1e-6, prec="fp64", **ov):
    n = len(d["q"])
    order = 2 if d["theta"] is not None else (1 if d["mu"] is not None else 0)
    pl = ak.Plan(n, 0.5 * d["edge"], eps, order, prec, far="fft", **ov)
    e, F, G = pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    pl.sync()
    return pl, e.item(), F.cpu().numpy(), G.cpu().numpy()


@pytest.mark.parametrize("depth,order,eq,kind,split", [(0, 4, 4, "qmt", False), (1, 4, 3, "qmt", False),
                                                       (2, 5, 5, "qmt", False), (2, 4, 6, "q", False),
                                                       (3, 4, 4, "qm", False), (1, 4, 4, "qmt", True),
                                                       (2, 5, 5, "qmt", True), (3, 4, 4, "qm", True)])
def test_fft_stage_parity_with_reference(ak, depth, order, eq, kind, split):
    """split: the cell transforms in the three passes that depths 5 and 6 use, forced at small depth."""
    d = _system(kind)
    pl, e, F, G = _run(ak, d, depth=depth, order=order, images=3, eq_order=eq, fft_split=split)
    st = pl.stats
    assert st["far_field"] == ak.ANKH_FAR_FFT and st["eq_order"] == eq and st["depth"] == depth
    assert st["fft_split"] == int(split)
    terms = pl.last_terms()
    r = ankh_ref.evaluate(d["pos"], d["q"], d["mu"], d["theta"], d["edge"], st["depth"], st["order"], st["xi"],
                          st["images"], grad=True, far="fft", eq_order=eq)
    scale = abs(r["e_near"]) + abs(r["e_self"]) + 1.0
    assert terms["periodic"] == 0.0
    assert abs(terms["far_levels"] - r["e_far_levels"][0]) <= 1e-12 * scale
    assert abs(terms["near"] - r["e_near"]) <= 1e-12 * scale
    assert abs(e - r["energy"]) <= 1e-12 * scale
    assert rel_rms(F, r["forces"]) <= 1e-11
    if d["mu"] is not None:
        assert rel_rms(G, r["dEdmu"]) <= 1e-11
    pl.close()


@pytest.mark.parametrize("leaves,order,eq,kind,split", [(3, 4, 4, "qmt", False), (5, 4, 4, "qm", False),
                                                        (6, 3, 5, "q", False), (12, 4, 4, "qm", False),
                                                        (12, 4, 4, "qmt", True)])
def test_fft_stage_parity_any_leaf_grid(ak, leaves, order, eq, kind, split):
    """A leaf grid that is not an octree level (3, 5, 6 per axis: direct DFTs along the cell axes; 12:
    the 4 x 3 two-phase transforms that 20 and 24 also use, all cells of a node frequency in one
    block, or in three passes through memory on request; lexicographic pair-kernel order) against the
    NumPy transcription on the same grid."""
    d = _system(kind)
    pl, e, F, G = _run(ak, d, leaves=leaves, order=order, images=3, eq_order=eq, fft_split=split)
    st = pl.stats
    assert st["leaves_per_axis"] == leaves and st["depth"] == -1
    if leaves == 12:
        assert st["fft_split"] == int(split)
    terms = pl.last_terms()
    r = ankh_ref.evaluate(d["pos"], d["q"], d["mu"], d["theta"], d["edge"], 0, st["order"], st["xi"],
                          st["images"], grad=True, far="fft", eq_order=eq, leaves=leaves)
    scale = abs(r["e_near"]) + abs(r["e_self"]) + 1.0
    assert abs(terms["far_levels"] - r["e_far_levels"][0]) <= 1e-12 * scale
    assert abs(terms["near"] - r["e_near"]) <= 1e-12 * scale
    assert abs(e - r["energy"]) <= 1e-12 * scale
    assert rel_rms(F, r["forces"]) <= 1e-11
    if d["mu"] is not None:
        assert rel_rms(G, r["dEdmu"]) <= 1e-11
    pl.close()


@pytest.mark.parametrize("leaves", [16, 20, 24])
def test_fft_water_288000_other_grids(ak, leaves):
    """The benchmark box on the 16^3 octree level (one-block cell transforms), on a 20^3 grid (4 x 5
    two-phase transforms, one block per node frequency) and on the planner's 24^3 grid (4 x 6, three
    passes in float64): FP64 against ANKH-FMM at depth 4 and the stored oracle atoms; mixed against
    FP64."""
    d = synth.workload("water_288000")
    n = len(d["q"])
    pl, e, F, G = _run(ak, d, eps=1e-6, leaves=leaves)
    assert pl.stats["leaves_per_axis"] == leaves
    pl.close()
    pm, em, Fm, Gm = _run(ak, d, eps=1e-6, prec="mixed_bf16x3", leaves=leaves)
    # the mixed modes: float32 transforms, in one block per node frequency on 24^3 (110 KB of LDS)
    assert pm.stats["far_precision"] == 1
    if leaves in (20, 24):
        assert pm.stats["fft_split"] == 0
    pm.close()
    pf = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64", far="fmm")
    ef, Ff, Gf = pf.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    pf.sync()
    ef, Ff, Gf = ef.item(), Ff.cpu().numpy(), Gf.cpu().numpy()
    pf.close()
    # smaller leaves hand more (and closer) pairs to the interpolated far field: at 24^3 the fields
    # of the two methods differ by ~3e-5 at the same order
    assert abs(e - ef) <= 1e-6 * abs(ef)
    assert rel_rms(F, Ff) <= 1e-5
    assert rel_rms(G, Gf) <= 5e-5
    assert abs(em - e) <= 1e-5 * abs(e)
    assert rel_rms(Fm, F) <= 1e-4 and rel_rms(Gm, G) <= 1e-4
    path = os.path.join(GOLDEN, "water_288000_sites.npz")
    if os.path.exists(path):
        g = np.load(path)
        sel = g["sel"]
        assert rel_rms(F[sel], g["forces"]) <= 1e-5
        assert rel_rms(G[sel], g["dEdmu"]) <= 1e-4
        assert rel_rms(Fm[sel], g["forces"]) <= 1e-4


def test_fft_20_cells_one_block_vs_three_passes(ak):
    """The 20^3 grid of the benchmark box with the cells of each node frequency in one block (where the
    device grants the 128 KB of LDS this takes) and in three passes: the same transform, so the two
    agree to rounding (the accuracy of this grid against the oracle: the full-size test)."""
    d = synth.workload("water_9000")
    res = {}
    for split in (False, True):
        pl, e, F, G = _run(ak, d, eps=1e-7, leaves=20, fft_split=split)
        st = pl.stats
        assert st["leaves_per_axis"] == 20
        if split:
            assert st["fft_split"] == 1
        res[split] = (e, F, G, st["fft_split"])
        pl.close()
    (e0, F0, G0, s0), (e1, F1, G1, _) = res[False], res[True]
    print(f"20^3 cell transforms: default path fft_split={s0}")
    assert abs(e0 - e1) <= 1e-12 * abs(e1)
    assert rel_rms(F0, F1) <= 1e-11 and rel_rms(G0, G1) <= 1e-11


def test_fft_water_9000_fp64_vs_oracle(ak):
    d = synth.workload("water_9000")
    g = np.load(os.path.join(GOLDEN, "water_9000.npz"))
    pl, e, F, G = _run(ak, d, eps=1e-7)
    assert abs(e - float(g["energy"])) <= 1e-6 * abs(float(g["energy"]))
    assert rel_rms(F, g["forces"]) <= 1e-5
    assert rel_rms(G, g["dEdmu"]) <= 1e-5
    pl.close()


def _away_from_faces(pos, edge, nside, h, count, seed):
    w = edge / nside
    x = pos + 0.5 * edge
    frac = (x / w) - np.floor(x / w)
    ok = np.all((frac * w > 20 * h) & ((1 - frac) * w > 20 * h), axis=1)
    idx = np.nonzero(ok)[0]
    return np.random.default_rng(seed).choice(idx, count, replace=False)


@pytest.mark.parametrize("leaves", [None, 5])
def test_fft_adjoint_is_gradient_of_energy(ak, leaves):
    d = synth.water(300, seed=21)
    n = len(d["q"])
    pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64", far="fft", leaves=leaves)
    pos, q, mu, th = T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"])
    _, F, G = pl.energy_forces(pos, q, mu, th)
    pl.sync()
    F = F.cpu().numpy()
    G = G.cpu().numpy()
    h = 1e-5
    for i in _away_from_faces(d["pos"], d["edge"], pl.stats["leaves_per_axis"], h, 4, 6):
        for c in range(3):
            vals = []
            for s in (+1, -1):
                p = pos.clone()
                p[i, c] += s * h
                vals.append(pl.energy(p, q, mu, th).item())
            assert -(vals[0] - vals[1]) / (2 * h) == pytest.approx(F[i, c], rel=1e-6, abs=1e-6 * np.abs(F).max())
            vals = []
            for s in (+1, -1):
                m = mu.clone()
                m[i, c] += s * h
                vals.append(pl.energy(pos, q, m, th).item())
            assert (vals[0] - vals[1]) / (2 * h) == pytest.approx(G[i, c], rel=1e-6, abs=1e-6 * np.abs(G).max())
    pl.close()


def test_fft_water_288000_full_size(ak):
    """The benchmark box on the planner's grid (24^3 leaves, 21 atoms each: the two-phase 4 x 6 cell
    transforms, in one block per node frequency in float32), the configuration bench.py times: FP64
    ANKH-FFT against ANKH-FMM and the stored oracle atoms; the mixed modes against FP64 ANKH-FFT.
    Smaller leaves hand closer pairs to the interpolated far field, so at 24^3 the fields of the two
    methods differ by ~3e-5 at the same order."""
    d = synth.workload("water_288000")
    out = {}
    for prec in ("fp64", "mixed", "mixed_bf16x3"):
        pl, e, F, G = _run(ak, d, eps=1e-6, prec=prec)
        assert pl.stats["leaves_per_axis"] == 24
        out[prec] = (e, F, G)
        pl.close()
    n = len(d["q"])
    pf = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64", far="fmm")
    ef, Ff, Gf = pf.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    pf.sync()
    ef, Ff, Gf = ef.item(), Ff.cpu().numpy(), Gf.cpu().numpy()
    pf.close()
    e64, F64, G64 = out["fp64"]
    assert abs(e64 - ef) <= 1e-6 * abs(ef)
    assert rel_rms(F64, Ff) <= 1e-5
    assert rel_rms(G64, Gf) <= 5e-5
    for prec in ("mixed", "mixed_bf16x3"):
        e, F, G = out[prec]
        assert abs(e - e64) <= 1e-5 * abs(e64)
        assert rel_rms(F, F64) <= 1e-4
        assert rel_rms(G, G64) <= 1e-4
    path = os.path.join(GOLDEN, "water_288000_sites.npz")
    if os.path.exists(path):
        g = np.load(path)
        sel = g["sel"]
        assert rel_rms(F64[sel], g["forces"]) <= 1e-5
        assert rel_rms(G64[sel], g["dEdmu"]) <= 1e-4


def test_fft_derivs_run_on_the_fft_far_field(ak):
    """ankh_energy_derivs evaluates through the same far field: its outputs agree with ANKH-FMM within
    the approximation error, on the same leaves (depth 1, the octree rule's choice for this box)."""
    d = synth.water(300, seed=5)
    n = len(d["q"])
    out = {}
    for far in ("fmm", "fft"):
        pl = ak.Plan(n, 0.5 * d["edge"], 1e-7, 2, "fp64", far=far, depth=1)
        o = pl.energy_derivs(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
        pl.sync()
        out[far] = {k: v.cpu().numpy() for k, v in o.items()}
        pl.close()
    for k in ("dEdq", "dEdtheta", "forces", "dEdmu"):
        assert rel_rms(out["fft"][k], out["fmm"][k]) <= 1e-5, k


def test_fft_depth_5_vs_fmm(ak):
    """Depth 5 (32^3 leaves: the cell transforms in three passes through HBM) on the benchmark box:
    ANKH-FFT against ANKH-FMM at the same depth, FP64; the mixed mode against FP64."""
    d = synth.workload("water_288000")
    n = len(d["q"])
    pl, e, F, G = _run(ak, d, eps=1e-6, depth=5)
    assert pl.stats["fft_split"] == 1
    pl.close()
    pm, em, Fm, Gm = _run(ak, d, eps=1e-6, prec="mixed_bf16x3", depth=5)
    pm.close()
    pf = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64", far="fmm", depth=5)
    ef, Ff, Gf = pf.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    pf.sync()
    ef, Ff, Gf = ef.item(), Ff.cpu().numpy(), Gf.cpu().numpy()
    pf.close()
    assert abs(e - ef) <= 1e-6 * abs(ef)
    assert rel_rms(F, Ff) <= 1e-5
    assert rel_rms(G, Gf) <= 2e-5
    assert abs(em - e) <= 1e-5 * abs(e)
    assert rel_rms(Fm, F) <= 1e-4 and rel_rms(Gm, G) <= 1e-4


def test_fft_depth_6_vs_fmm(ak):
    """The 3,000,000-molecule box at its automatic depth 6 (64^3 leaves), ANKH-FFT against ANKH-FMM
    (FP64, accuracy 1e-5)."""
    d = synth.workload("water_9000000")
    n = len(d["q"])
    out = {}
    for far in ("fft", "fmm"):
        pl = ak.Plan(n, 0.5 * d["edge"], 1e-5, 2, "fp64", far=far)
        assert pl.stats["depth"] == 6
        e, F, G = pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
        pl.sync()
        out[far] = (e.item(), F.cpu().numpy(), G.cpu().numpy())
        pl.close()
        del e, F, G
        torch.cuda.empty_cache()
    (e1, F1, G1), (e2, F2, G2) = out["fft"], out["fmm"]
    assert abs(e1 - e2) <= 1e-5 * abs(e2)
    assert rel_rms(F1, F2) <= 1e-4 and rel_rms(G1, G2) <= 1e-4


def test_fft_planning_errors(ak):
    d = synth.water(100, seed=4)
    n = len(d["q"])
    for kw in (dict(depth=7), dict(eq_order=11), dict(eq_order=1)):
        with pytest.raises(ak.AnkhError) as ei:
            ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, "fp64", far="fft", **kw)
        assert ei.value.status == 1, kw
    # the automatic grid of ANKH-FFT: about 0.17 n_u atoms per leaf on a grid with fast transforms
    # (2,000,000 atoms at order 6: 32^3); beyond 16 leaves per axis the cell transforms run in three passes
    pl = ak.Plan(2_000_000, 100.0, 1e-6, 2, "mixed", far="fft")
    assert pl.stats["depth"] == 5 and pl.stats["far_field"] == ak.ANKH_FAR_FFT and pl.stats["fft_split"] == 1
    pl.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fft_overlap_matches_one_stream(ak, prec):
    """The far-field chain on the plan's second stream beside the pair kernel gives bitwise the result of
    the one-stream schedule (every kernel writes its own outputs; the sums run in a fixed order).  Stage
    timing mode 2 keeps the overlap and times the cell transforms and the pair kernel."""
    d = synth.workload("water_9000")
    n = len(d["q"])
    outs = []
    for overlap in (True, False):
        pl = ak.Plan(n, 0.5 * d["edge"], 1e-6, 2, prec, far="fft", leaves=16, overlap=overlap)
        assert pl.stats["overlap"] == int(overlap) and pl.stats["leaves_per_axis"] == 16
        e, F, G = pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
        pl.sync()
        outs.append((e.item(), F.cpu().numpy(), G.cpu().numpy()))
        if overlap:
            pl.set_timing(2)
            for _ in range(3):
                pl.energy_forces(T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
            st = pl.get_stats()
            assert st["timed_evals"] == 3
            assert 0 < st["stage_ms"]["p2p"] < 50 and 0 < st["stage_ms"]["m2l"] < 50
        pl.close()
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])

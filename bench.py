"""Benchmark of the interpolated-Ewald hot path on one MI355X.

One step = one energy + forces + fields evaluation (the whole hot path:
sort, P2M, the far field, L2P, P2P, reductions) of the synthetic water box
of 96,000 rigid 3-site molecules
(288,000 atoms, edge 142.18 A, charges + dipoles + quadrupoles), inputs
resident in HBM.  The mixed-precision path is the headline; the FP64 path is
timed on the same inputs and plan parameters for the speed-up and the
accuracy of the mixed path, and both are compared with the stored
classical-Ewald oracle values.  The far field is ANKH-FFT by default (forward
node transform, cell FFTs with the spectrum, inverse node transform); with
--far fmm it is the multilevel chain (M2M, M2L on every level, far-image root
operator, L2L).  The other method is timed on the same input for comparison
(its M2L contraction gives the matrix-core roofline).

Two more workloads are timed as sub-records: the 1,000,000-ion melt (mixed
energy + forces) and the 9,000,000-atom water box (mixed and FP64 energy +
forces + fields in one pass, checked on its 20,000-atom cut-out against the
oracle).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "E+forces evals/s per atom on 1 MI355X, mixed vs FP64, rel RMS force err"
GOLDEN = os.path.join(ROOT, "tests", "golden")

# Algorithmic flops of the near field per UNORDERED pair of atoms (the mutual
# form evaluates each pair once), counted term by term from the pair kernel's
# formula (FMA = 2, add / mul = 1, erfc / exp / rsqrt = 1 each), keyed by
# (moment order, forces, fields):
#  - charges + dipoles + quadrupoles with the energy, the force and the field at
#    both atoms: 300;
#  - charges + dipoles with the energy and the force: 83 (r^2, 1/r, 1/r^2, r: 8;
#    B0 and the Gaussian: 5; B1..B3: 11; dipole invariants and c0..c2: 21;
#    energy: 6; a1, a2: 6; sum c_n B_{n+1}: 5; force: 15; into both atoms: 6).
P2P_FLOP_PER_UNORDERED_PAIR = {(2, True, True): 300.0, (1, True, False): 83.0}

# HBM traffic of one P2P launch measured with rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE, calibrated against a copy of known size) for the kernel source
# with the recorded SHA-256; reported only while the source is unchanged.
P2P_COUNTERS = os.path.join(ROOT, "profiles", "p2p_water_288000_counters.txt")
P2P_SOURCE = os.path.join(ROOT, "paper_2212_08284_amd", "csrc", "ankh_p2p.hip")
FFT_COUNTERS = os.path.join(ROOT, "profiles", "fft_cells_water_288000_counters.txt")
FFT_SOURCE = os.path.join(ROOT, "paper_2212_08284_amd", "csrc", "ankh_fft.hip")
M2L_COUNTERS = os.path.join(ROOT, "profiles", "m2l_water_288000_counters.txt")
M2L_SOURCES = [os.path.join(ROOT, "paper_2212_08284_amd", "csrc", f) for f in ("ankh_m2l.hip", "ankh_compress.hip")]

PEAK = {  # MI355X, TFLOP/s (hbm: GB/s)
    "hbm": 8000.0,
    "valu_fp64": 78.6,           # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
    "valu_fp32": 157.3,          # the published FP32 vector peak (packed FP32, two lanes per instruction)
    "valu_fp32_unpacked": 78.6,  # one FP32 FMA per lane and cycle: the rate of the instructions issued here
    "mfma_fp64": 78.6,
    "mfma_fp32": 157.3,
    "mfma_bf16": 2500.0,
}
PREC_NAME = {0: "f64", 1: "f32", 2: "bf16x3"}


def counter_traffic(counters=P2P_COUNTERS, source=P2P_SOURCE, leaves=None, suffix=""):
    """Calibrated HBM bytes per launch of a kernel (or stage) from its committed counter summary, or None
    when the summary is missing, the kernel source (one file, or several hashed in order as one stream)
    has changed since, or it was taken on another leaf grid."""
    import hashlib
    try:
        rec = {}
        with open(counters) as fh:
            for ln in fh:
                if "=" in ln and not ln.lstrip().startswith("#"):
                    k, v = ln.split("=", 1)
                    rec[k.strip()] = v.strip()
        h = hashlib.sha256()
        for src in ([source] if isinstance(source, str) else source):
            with open(src, "rb") as fh:
                h.update(fh.read())
        sha = h.hexdigest()
        if rec.get("kernel_source_sha256") != sha:
            return None
        if leaves is not None and rec.get("leaves_per_axis") != str(leaves):
            return None
        return float(rec["fetch_bytes_per_launch" + suffix]) + float(rec["write_bytes_per_launch" + suffix])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def err_stats(a, ref):
    """relative RMS, and the per-atom relative errors |a_i - ref_i| / |ref_i| (max and median)"""
    d = np.linalg.norm(a - ref, axis=1)
    r = np.linalg.norm(ref, axis=1)
    per = d / np.maximum(r, 1e-300)
    return {"rel_rms": float(np.sqrt(np.sum(d ** 2) / np.sum(r ** 2))), "max_atom_rel": float(per.max()),
            "median_atom_rel": float(np.median(per))}


def golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    return np.load(path) if os.path.exists(path) else None


def dtype_name(st):
    near, far = PREC_NAME[st["near_precision"]], PREC_NAME[st["far_precision"]]
    if near == far:
        return near
    return f"{near} near field + {far} far field ({'ANKH-FFT' if st['far_field'] == 2 else 'ANKH-FMM'})"


def timed_run(plan, args_dev, steps, warmup, torch, fields=True):
    """K timed steps with hipEvents around the far-field contraction and pair-kernel stages only (every event
    idles the device for a few microseconds); then K more steps with an event at every stage boundary for the
    stage breakdown.  Returns (seconds per step, stats of the timed steps, breakdown, outputs)."""
    for _ in range(warmup):
        plan.energy_forces(*args_dev, fields=fields)
    torch.cuda.synchronize()
    plan.set_timing(2)
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = plan.energy_forces(*args_dev, fields=fields)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    stats = plan.get_stats()
    plan.set_timing(1)
    for _ in range(steps):
        plan.energy_forces(*args_dev, fields=fields)
    breakdown = plan.get_stats()["stage_ms"]
    plan.set_timing(0)
    plan.sync()
    return dt, stats, breakdown, out


def p2p_roofline(st, breakdown, key, leaves=None, traffic=True):
    """The pair kernel against the FP32 vector peak: algorithmic flops per launch over its average hipEvent
    duration in the timed steps (and alone, in the breakdown pass)."""
    sm = st["stage_ms"]
    unordered = st["near_pairs"] / 2.0
    fpp = P2P_FLOP_PER_UNORDERED_PAIR[key]
    flops = unordered * fpp
    peak = PEAK["valu_fp32"] if st["near_precision"] == 1 else PEAK["valu_fp64"]
    tf = flops / (sm["p2p"] * 1e-3) / 1e12
    alone = flops / (breakdown["p2p"] * 1e-3) / 1e12
    rec = {"kernel": "p2p", "bound": "alu", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
           "traffic": counter_traffic(leaves=leaves) if traffic else None,
           "flop_per_launch": flops, "unordered_pairs": unordered, "flop_per_unordered_pair": fpp,
           "avg_launch_ms": sm["p2p"], "alone_avg_launch_ms": breakdown["p2p"], "alone_achieved": alone,
           "alone_frac": alone / peak}
    if st["near_precision"] == 1:
        rec["frac_of_unpacked_fp32"] = tf / PEAK["valu_fp32_unpacked"]
        rec["alone_frac_of_unpacked_fp32"] = alone / PEAK["valu_fp32_unpacked"]
        rec["note"] = ("peak = the published FP32 vector rate, 157.3 TFLOP/s (packed FP32, two lanes per "
                       "instruction); this build issues unpacked FP32 (one FMA per lane and cycle, 78.6 TFLOP/s: "
                       "frac_of_unpacked_fp32).  alone_*: the breakdown pass (an event at every stage boundary)")
    return rec


def m2l_roofline(st, breakdown, mode):
    """The ANKH-FMM M2L contraction (stage 4) against the matrix-core peak of its datatype: algorithmic flops
    (2 * 189 * r_e^2 per cell of level e, plus the basis change of compressed levels) over the stage time."""
    flops = st["m2l_flops"]
    peak = PEAK["mfma_bf16"] if mode == "mixed_bf16x3" else (PEAK["mfma_fp32"] if mode == "mixed" else
                                                            PEAK["mfma_fp64"])
    t = st["stage_ms"]["m2l"]
    tf = flops / (t * 1e-3) / 1e12
    alone = flops / (breakdown["m2l"] * 1e-3) / 1e12
    traffic = (counter_traffic(M2L_COUNTERS, M2L_SOURCES, st.get("leaves_per_axis"),
                               "" if mode == "mixed_bf16x3" else "_f32")
               if mode in ("mixed_bf16x3", "mixed") else None)
    rec = {"kernel": "m2l", "bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
           "traffic": traffic, "flop_per_launch": flops, "avg_launch_ms": t, "alone_avg_launch_ms": breakdown["m2l"],
           "alone_achieved": alone, "alone_frac": alone / peak, "ranks": st.get("m2l_rank"),
           "note": "ANKH-FMM far-field contraction, all levels with the projection / expansion of compressed levels "
                   "(stage 4); algorithmic flops per cell of level e: 2 * 189 * r_e^2 (r_e the kept rank) + "
                   "4 * n_u * r_e for the basis change"}
    if mode == "mixed_bf16x3":
        rec["issued_frac"] = 3 * tf / peak
        rec["note"] += "; the split-precision product issues three bf16 products per algorithmic one (issued_frac)"
    if mode in ("mixed_bf16x3", "mixed"):
        rec["note"] += "; traffic: the counters' HBM bytes summed over the stage's launches"
    return rec


def fft_roofline(st, breakdown):
    """The ANKH-FFT cell transforms (stage 4) against the HBM peak: 16 B read + 16 B written of spectrum and
    the real spectrum read per kept node frequency and leaf (algorithmic bytes)."""
    sm = st["stage_ms"]
    pa = 2 * st["eq_order"] - 1
    nf = pa * pa * (pa // 2 + 1)
    nleaf = st["leaves_per_axis"] ** 3
    cb = 8 if st["far_precision"] == 0 else 4
    per = 4 * cb + cb
    nbytes = float(per * nf * nleaf)
    gbs = nbytes / (sm["m2l"] * 1e-3) / 1e9
    alone = nbytes / (breakdown["m2l"] * 1e-3) / 1e9
    return {"kernel": "fft_cells", "bound": "hbm", "achieved": gbs, "peak": PEAK["hbm"], "unit": "GB/s",
            "frac": gbs / PEAK["hbm"],
            "traffic": counter_traffic(FFT_COUNTERS, FFT_SOURCE, st["leaves_per_axis"]),
            "bytes_per_launch": nbytes, "avg_launch_ms": sm["m2l"], "alone_avg_launch_ms": breakdown["m2l"],
            "alone_achieved": alone, "alone_frac": alone / PEAK["hbm"], "passes": 3 if st["fft_split"] else 1,
            "note": f"ANKH-FFT cell transforms (stage 4): {nf} kept node frequencies x {nleaf} leaves, each read and "
                    f"written once as a complex {'float64' if cb == 8 else 'float32'} value and multiplied by the "
                    "real spectrum: the algorithmic bytes; traffic is the counters' sum over the stage's launches"}


def oracle_errors(E, F, G, name):
    """Errors of one evaluation against the stored oracle values of a workload (energy when stored; forces and
    fields of the stored atoms)."""
    out = {}
    ge = golden(f"{name}_energy")
    if ge is not None:
        out["rel_energy_err"] = float(abs(E - float(ge["energy"])) / abs(float(ge["energy"])))
    gs = golden(f"{name}_sites")
    if gs is not None:
        sel = gs["sel"]
        out["sites"] = int(len(sel))
        out["forces"] = err_stats(F[sel], gs["forces"])
        if G is not None:
            out["fields"] = err_stats(G[sel], gs["dEdmu"])
    return out


def induce_run(plan, args_dev, alpha, tol, torch, dev, reps=3):
    """Induced dipoles of the water polarisabilities: wall time of whole solves (the permanent
    field, the conjugate-gradient products, the final energy and forces), inputs resident."""
    a = torch.tensor(alpha, dtype=torch.float64, device=dev)
    plan.induce(*args_dev, a, tol=tol, forces=True)            # warm-up (allocates the solver vectors)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mi, e, F, it, r = plan.induce(*args_dev, a, tol=tol, forces=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    return {"tol": tol, "iterations": it, "rel_residual": r, "ms": ms, "ms_per_product": ms / (it + 2),
            "polarisabilities_A3": {"O": float(alpha[0]), "H": float(alpha[1])},
            "note": "one solve = the permanent field + one dipole-field evaluation per iteration + the final "
                    "energy and forces (it + 2 evaluations)", "_mu": mi.cpu().numpy()}


def derivs_run(plan, args_dev, torch, reps=5):
    """Wall time of one evaluation with every derivative (forces, fields, dE/dq, dE/dTheta) against
    energy + forces + fields alone; returns the outputs of the last call too."""
    plan.energy_derivs(*args_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = plan.energy_derivs(*args_dev)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    return {"ms_all_derivs": ms, "reps": reps,
            "note": "energy, forces, dE/dmu, dE/dq and dE/dTheta in one call (ankh_energy_derivs); the "
                    "charge and quadrupole derivatives add a gather-form pass over the near pairs and one over "
                    "the atoms"}, out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(data, eps, single_thread_water=False):
    """The classical-Ewald oracle timed on this host's cores: on a bounded cut-out of the benchmark box
    (the value), and on the 1000-charge box and the 9000-atom water box in full."""
    import oracle
    import synth
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sub_edge = (2000 / synth.WATER_DENSITY) ** (1.0 / 3.0)     # ~2000 molecules, same density
    cut = synth.water_cutout(data, sub_edge)
    n = len(cut["q"])
    t0 = time.perf_counter()
    oracle.ewald(cut["pos"], cut["q"], cut["mu"], cut["theta"], edge=cut["edge"], eps=eps, nthreads=nthreads)
    dt = time.perf_counter() - t0
    full = {}
    d1 = synth.workload("charges_1000")
    for nt in (nthreads, 1):
        t0 = time.perf_counter()
        oracle.ewald(d1["pos"], d1["q"], edge=d1["edge"], eps=1e-8, grad=True, nthreads=nt)
        full[f"charges_1000_threads{nt}_s"] = time.perf_counter() - t0
    d2 = synth.workload("water_9000")
    for nt in ((nthreads, 1) if single_thread_water else (nthreads,)):
        t0 = time.perf_counter()
        oracle.ewald(d2["pos"], d2["q"], d2["mu"], d2["theta"], edge=d2["edge"], eps=eps, grad=True, nthreads=nt)
        full[f"water_9000_threads{nt}_s"] = time.perf_counter() - t0
    full["note"] = ("whole classical-Ewald solutions: the 1000-charge box (energy + forces, accuracy 1e-8) and the "
                    f"9000-atom water box (energy + forces + fields, accuracy {eps:g}); seconds of wall time")
    return {"value": n / dt, "unit": "atoms*evals/s", "cores": nthreads, "kind": "oracle",
            "sample": f"classical-Ewald oracle, energy+forces+fields, on a periodic cut-out of {n} atoms "
                      f"(whole molecules, edge {cut['edge']:.2f} A) of the benchmark box, accuracy {eps:g}; "
                      f"{dt:.2f} s wall; Ewald cost grows as N^1.5, so per-atom throughput at 288,000 atoms "
                      f"would be lower",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(), "full_configs": full}


def sub_ionic(ak, args, torch, dev, T):
    """The 1,000,000-ion melt (charges + dipoles): mixed energy + forces, the pair-kernel roofline, and the
    errors against the stored oracle ions."""
    import synth
    d = synth.workload("ionic_1000000")
    n = len(d["q"])
    a = (T(d["pos"]), T(d["q"]), T(d["mu"]), None)
    pl = ak.Plan(n, 0.5 * d["edge"], args.eps, 1, args.mode)
    t, st, bd, out = timed_run(pl, a, args.steps, args.warmup, torch, fields=False)
    E, F = out[0].item(), out[1].cpu().numpy()
    pl.close()
    rec = {"workload": "ionic_1000000: 1,000,000 +-1 charges with dipoles, 0.1 atoms/A^3, energy+forces",
           "n_atoms": n, "edge_A": d["edge"], "mode": args.mode, "dtype": dtype_name(st),
           "ms_per_step": t * 1e3, "value": n / t, "unit": "atoms*evals/s", "far_field": st["far_field"],
           "leaves_per_axis": st["leaves_per_axis"], "order": st["order"], "stage_ms": bd,
           "roofline": p2p_roofline(st, bd, (1, True, False), traffic=False),
           "vs_oracle": oracle_errors(E, F, None, "ionic_1000000")}
    del a, out
    torch.cuda.empty_cache()
    return rec


def sub_octupole(ak, args, torch, dev, T, data):
    """The benchmark box with a traceless octupole on every atom as well (ankh_energy_octupole, the next
    order of the operator D): mixed and FP64 energy + forces + fields, and the mixed path against FP64.
    (Parity with the oracle's octupoles is a test: classical Ewald with octupoles is too slow at this size.)"""
    import synth
    n = len(data["q"])
    om = synth.water_octupoles(n // 3, seed=5)
    a = (T(data["pos"]), T(data["q"]), T(data["mu"]), T(data["theta"]), T(om))
    rec = {"workload": "water_288000 with octupoles: q+mu+Theta+Omega, energy+forces+fields", "n_atoms": n}
    outs = {}
    for key, mode in (("mixed", args.mode), ("fp64", "fp64")):
        pl = ak.Plan(n, 0.5 * data["edge"], args.eps, 3, mode)
        for _ in range(args.warmup):
            pl.energy_octupole(*a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = pl.energy_octupole(*a)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        pl.set_timing(1)
        for _ in range(args.steps):
            pl.energy_octupole(*a)
        st = pl.get_stats()
        pl.close()
        rec[key] = {"ms_per_step": t * 1e3, "value": n / t, "unit": "atoms*evals/s", "dtype": dtype_name(st),
                    "stage_ms": st["stage_ms"]}
        outs[key] = (out[0].item(), out[1].cpu().numpy(), out[2].cpu().numpy())
    (e0, F0, G0), (e1, F1, G1) = outs["fp64"], outs["mixed"]
    rec["speedup_mixed_vs_fp64"] = rec["fp64"]["ms_per_step"] / rec["mixed"]["ms_per_step"]
    rec["mixed_vs_fp64"] = {"rel_energy_err": abs(e1 - e0) / abs(e0), "rel_rms_force_err": rel_rms(F1, F0),
                            "rel_rms_field_err": rel_rms(G1, G0)}
    del a
    torch.cuda.empty_cache()
    return rec


def sub_water9m(ak, args, torch, dev, T):
    """The 9,000,000-atom water box: mixed and FP64 energy + forces + fields in one pass, the speed-up, and the
    20,000-atom corner cut-out against the stored oracle solution."""
    import synth
    d = synth.workload("water_9000000")
    n = len(d["q"])
    a = (T(d["pos"]), T(d["q"]), T(d["mu"]), T(d["theta"]))
    rec = {"workload": "water_9000000: 3,000,000 rigid 3-site molecules, q+mu+Theta, energy+forces+fields",
           "n_atoms": n, "edge_A": d["edge"]}
    outs = {}
    for prec in (args.mode, "fp64"):
        pl = ak.Plan(n, 0.5 * d["edge"], args.eps, 2, prec)
        t, st, bd, out = timed_run(pl, a, args.steps, args.warmup, torch)
        outs[prec] = [x.cpu().numpy() for x in out]
        key = "mixed" if prec != "fp64" else "fp64"
        rec[key] = {"ms_per_step": t * 1e3, "value": n / t, "dtype": dtype_name(st), "far_field": st["far_field"],
                    "leaves_per_axis": st["leaves_per_axis"], "order": st["order"], "plan_ms": st["plan_ms"],
                    "stage_ms": bd, "roofline": p2p_roofline(st, bd, (2, True, True), traffic=False)}
        pl.close()
        del out
        torch.cuda.empty_cache()
    rec["speedup_mixed_vs_fp64"] = rec["fp64"]["ms_per_step"] / rec["mixed"]["ms_per_step"]
    m, f = outs[args.mode], outs["fp64"]
    rec["mixed_vs_fp64"] = {"rel_energy_err": float(abs(m[0][0] - f[0][0]) / abs(f[0][0])),
                            "forces": err_stats(m[1], f[1]), "fields": err_stats(m[2], f[2])}
    del a, outs
    torch.cuda.empty_cache()
    g = golden("water_cutout_20k")
    if g is not None:
        c = synth.water_cutout(d, 58.442)
        nc = len(c["q"])
        ca = (T(c["pos"]), T(c["q"]), T(c["mu"]), T(c["theta"]))
        cut = {"n_atoms": nc, "edge_A": c["edge"]}
        for prec in (args.mode, "fp64"):
            pl = ak.Plan(nc, 0.5 * c["edge"], args.eps, 2, prec)
            e, F, G = pl.energy_forces(*ca)
            pl.sync()
            pl.close()
            cut["mixed" if prec != "fp64" else "fp64"] = {
                "rel_energy_err": float(abs(e.item() - float(g["energy"])) / abs(float(g["energy"]))),
                "forces": err_stats(F.cpu().numpy(), g["forces"]), "fields": err_stats(G.cpu().numpy(), g["dEdmu"])}
        rec["cutout_vs_oracle"] = cut
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water_288000")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-single-thread-water", action="store_true",
                    help="skip the one-thread oracle run on the 9000-atom water box (about 100 s)")
    ap.add_argument("--mixed-only", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--mode", default="mixed_bf16x3", choices=["mixed", "mixed_bf16x3"],
                    help="precision mode of the headline (mixed) path")
    ap.add_argument("--no-induce", action="store_true", help="skip the induced-dipole solve")
    ap.add_argument("--no-derivs", action="store_true", help="skip the charge / quadrupole derivative timing")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1,000,000-ion, 9,000,000-atom and octupole sub-records")
    ap.add_argument("--induce-tol", type=float, default=1e-6)
    ap.add_argument("--far", default="fft", choices=["fmm", "fft"],
                    help="far-field method of the timed path: ANKH-FFT (the variant the paper times) or "
                         "ANKH-FMM (multilevel M2L)")
    ap.add_argument("--depth", type=int, default=None, help="octree depth (default: the planner's choice)")
    ap.add_argument("--leaves", type=int, default=None,
                    help="ANKH-FFT leaves per axis (any count up to 40, or a power of two; default 2^depth)")
    ap.add_argument("--overlap", default="auto", choices=["auto", "on", "off"],
                    help="far-field chain beside the pair kernel on a second stream (auto: the plan's choice)")
    ap.add_argument("--no-far-compare", action="store_true",
                    help="skip timing the other far-field method on the same input")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the timed region, one device-to-device copy of this many MiB (a plain copy kernel "
                         "of known size that calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU sharding is a "
              f"design only", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2212_08284_amd as ak
    import synth

    data = synth.workload(args.workload)
    n = len(data["q"])
    dev = torch.device("cuda:0")

    def T(a):
        return None if a is None else torch.tensor(a, dtype=torch.float64, device=dev)

    args_dev = (T(data["pos"]), T(data["q"]), T(data["mu"]), T(data["theta"]))
    if args.calib_copy_mb > 0:
        nb = args.calib_copy_mb << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb} bytes read, {nb} bytes written")
        del src, dst
    rB = 0.5 * data["edge"]
    log(f"workload {args.workload}: n={n} edge={data['edge']:.3f}")

    ovl = {"auto": None, "on": True, "off": False}[args.overlap]
    lv = args.leaves if args.far == "fft" else None
    pm = ak.Plan(n, rB, args.eps, 2, args.mode, far=args.far, overlap=ovl, depth=args.depth, leaves=lv)
    log(f"mixed plan: {pm.stats}")
    t_mixed, st_mixed, bd_mixed, out_mixed = timed_run(pm, args_dev, args.steps, args.warmup, torch)
    log(f"mixed: {t_mixed * 1e3:.3f} ms/step timed stages {st_mixed['stage_ms']} breakdown {bd_mixed}")
    Em, Fm, Gm = [x.double().cpu().numpy() for x in out_mixed]

    far_other = None
    roof_m2l = None
    roof_m2l_f32 = None
    if not args.no_far_compare:
        alt = "fft" if args.far == "fmm" else "fmm"
        pa = ak.Plan(n, rB, args.eps, 2, args.mode, far=alt, overlap=ovl, depth=args.depth)
        t_a, st_a, bd_a, out_a = timed_run(pa, args_dev, args.steps, args.warmup, torch)
        Ea, Fa, Ga = [x.double().cpu().numpy() for x in out_a]
        far_other = {"far": alt, "ms_per_step": t_a * 1e3, "value": n / t_a, "plan_ms": st_a["plan_ms"],
                     "depth": st_a["depth"], "eq_order": st_a["eq_order"], "dtype": dtype_name(st_a), "stage_ms": bd_a,
                     "rel_energy_diff": float(abs(Ea[0] - Em[0]) / abs(Em[0])),
                     "rel_rms_force_diff": rel_rms(Fa, Fm), "rel_rms_field_diff": rel_rms(Ga, Gm)}
        if alt == "fmm":
            roof_m2l = m2l_roofline(st_a, bd_a, args.mode)
        pa.close()
        log(f"{alt}: {far_other}")
        if alt == "fmm" and args.mode != "mixed":
            # the same ANKH-FMM contraction on the float32 matrix cores (ANKH_MIXED): its own peak
            pf32 = ak.Plan(n, rB, args.eps, 2, "mixed", far="fmm", overlap=ovl, depth=args.depth)
            t_f, st_f, bd_f, _ = timed_run(pf32, args_dev, args.steps, args.warmup, torch)
            far_other["mixed_fp32_mfma"] = {"ms_per_step": t_f * 1e3, "value": n / t_f, "stage_ms": bd_f}
            roof_m2l_f32 = m2l_roofline(st_f, bd_f, "mixed")
            pf32.close()
    if args.far == "fmm":
        roof_m2l = m2l_roofline(st_mixed, bd_mixed, args.mode)

    derivs = None
    if not args.no_derivs:
        derivs, dmix = derivs_run(pm, args_dev, torch)
        derivs["ms_energy_forces_fields"] = t_mixed * 1e3
        log(f"derivs: {derivs}")

    induce = None
    if not args.no_induce and args.workload.startswith("water"):
        induce = induce_run(pm, args_dev, synth.water_polarisabilities(n // 3), args.induce_tol, torch, dev)
        log(f"induce: { {k: v for k, v in induce.items() if k != '_mu'} }")

    vs_oracle = {"mixed": oracle_errors(float(Em[0]), Fm, Gm, args.workload)}
    res = {}
    if not args.mixed_only:
        pf = ak.Plan(n, rB, args.eps, 2, "fp64", far=args.far, overlap=ovl, depth=args.depth, leaves=lv)
        t_fp64, st_fp64, bd_fp64, out_fp64 = timed_run(pf, args_dev, args.steps, args.warmup, torch)
        if derivs is not None:
            d64, dfp = derivs_run(pf, args_dev, torch)
            derivs["fp64"] = {"ms_all_derivs": d64["ms_all_derivs"], "ms_energy_forces_fields": t_fp64 * 1e3}
            derivs["mixed_vs_fp64"] = {
                "rel_rms_dEdq": rel_rms(dmix["dEdq"].cpu().numpy(), dfp["dEdq"].cpu().numpy()),
                "rel_rms_dEdtheta": rel_rms(dmix["dEdtheta"].cpu().numpy(), dfp["dEdtheta"].cpu().numpy())}
        if induce is not None:
            ind64 = induce_run(pf, args_dev, synth.water_polarisabilities(n // 3), args.induce_tol, torch, dev,
                               reps=1)
            induce["fp64"] = {k: ind64[k] for k in ("ms", "iterations", "ms_per_product")}
            induce["mixed_vs_fp64_rel_rms_mu_ind"] = rel_rms(induce.pop("_mu"), ind64.pop("_mu"))
            induce.pop("_mu", None)
        log(f"fp64: {t_fp64 * 1e3:.3f} ms/step breakdown {bd_fp64}")
        Ef, Ff, Gf = [x.double().cpu().numpy() for x in out_fp64]
        vs_oracle["fp64"] = oracle_errors(float(Ef[0]), Ff, Gf, args.workload)
        res = {
            "fp64_ms_per_step": t_fp64 * 1e3,
            "fp64_value": n / t_fp64,
            "fp64_dtype": dtype_name(st_fp64),
            "speedup_mixed_vs_fp64": t_fp64 / t_mixed,
            "mixed_vs_fp64": {"rel_energy_err": float(abs(Em[0] - Ef[0]) / abs(Ef[0])),
                              "rel_rms_force_err": rel_rms(Fm, Ff), "rel_rms_field_err": rel_rms(Gm, Gf),
                              "forces": err_stats(Fm, Ff), "fields": err_stats(Gm, Gf)},
            "fp64_stage_ms": bd_fp64,
            "fp64_roofline": p2p_roofline(st_fp64, bd_fp64, (2, True, True), traffic=False),
        }
        pf.close()
    log(f"vs oracle: {vs_oracle}")

    # roofline of the dominant kernel of the timed (mixed) path, from the live hipEvent stage timings
    sm = st_mixed["stage_ms"]
    roof_p2p = p2p_roofline(st_mixed, bd_mixed, (2, True, True), leaves=st_mixed["leaves_per_axis"])
    roof_far = fft_roofline(st_mixed, bd_mixed) if args.far == "fft" else roof_m2l
    roof = roof_p2p if sm["p2p"] >= sm["m2l"] else roof_far

    line = {
        "metric": METRIC,
        "value": n / t_mixed,
        "unit": "atoms*evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name(st_mixed),
        "mode": args.mode,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: rigid 3-site water, q+mu+Theta, energy+forces+fields",
                   "n_atoms": n, "edge_A": data["edge"], "rel_accuracy": args.eps,
                   "depth": st_mixed["depth"], "order": st_mixed["order"], "images": st_mixed["images"],
                   "xi": st_mixed["xi"], "far_field": args.far, "eq_order": st_mixed["eq_order"],
                   "leaves_per_axis": st_mixed["leaves_per_axis"],
                   "overlap": bool(st_mixed["overlap"]),
                   "parallelism": "single GPU"},
        "plan_ms": st_mixed["plan_ms"],
        "evals_per_s": 1.0 / t_mixed,
        "ns_per_day_equiv_dt2fs": 86400.0 / t_mixed * 2e-6,
        "stage_ms": bd_mixed,
        "stage_ms_note": "a separate pass of the same number of steps with an event at every stage boundary and the "
                         "stages in sequence on one stream; the timed steps carry events around stage 4 (the M2L, "
                         "or the cell transforms of ANKH-FFT) and the pair kernel only (and the far-field chain on a "
                         "second stream beside the pair kernel with --overlap on).  ANKH-FFT stages: m2m = forward node transform, m2l = cell transforms "
                         "with the spectrum, l2l = inverse node transform + leaf energies, periodic = none",
        "roofline": roof,
    }
    if roof is not roof_p2p:
        line["roofline_p2p"] = roof_p2p
    if args.far == "fft" and roof is not roof_far:
        line["roofline_fft_cells"] = roof_far
    if roof_m2l is not None:
        line["roofline_m2l"] = roof_m2l
    if roof_m2l_f32 is not None:
        line["roofline_m2l_fp32"] = roof_m2l_f32
    line.update(res)
    line["vs_oracle"] = vs_oracle
    if far_other is not None:
        line["far_other"] = far_other
    if derivs is not None:
        line["derivs"] = derivs
    if induce is not None:
        induce.pop("_mu", None)
        line["induce"] = induce
    pm.close()
    del args_dev, out_mixed
    torch.cuda.empty_cache()
    if not args.no_configs:
        line["configs"] = {}
        line["configs"]["ionic_1000000"] = sub_ionic(ak, args, torch, dev, T)
        log(f"ionic_1000000: {line['configs']['ionic_1000000']}")
        line["configs"]["water_9000000"] = sub_water9m(ak, args, torch, dev, T)
        log(f"water_9000000: {line['configs']['water_9000000']}")
        if data.get("theta") is not None:
            line["configs"]["water_288000_octupoles"] = sub_octupole(ak, args, torch, dev, T, data)
            log(f"octupoles: {line['configs']['water_288000_octupoles']}")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(data, args.eps, not args.no_cpu_single_thread_water)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

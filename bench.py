"""Benchmark of the interpolated-Ewald hot path on one MI355X.

One step = one energy + forces + fields evaluation (the whole hot path:
sort, P2M, the far field, L2P, P2P, reductions) of the synthetic water box
of 96,000 rigid 3-site molecules
(288,000 atoms, edge 142.18 A, charges + dipoles + quadrupoles), inputs
resident in HBM.  The mixed-precision path is the headline; the FP64 path is
timed on the same inputs and plan parameters for the speed-up and the
accuracy of the mixed path.  The far field is ANKH-FFT by default (forward
node transform, cell FFTs with the spectrum, inverse node transform); with
--far fmm it is the multilevel chain (M2M, M2L on every level, far-image root
operator, L2L).  The other method is timed on the same input for comparison.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "E+forces evals/s per atom on 1 MI355X, mixed vs FP64, rel RMS force err"

# Algorithmic flops of the near field per UNORDERED pair of atoms (the mutual
# form evaluates each pair once): the pair kernel's formula for charges +
# dipoles + quadrupoles with the energy, the force, the field at both atoms and
# the accumulation into both atoms, counted term by term from its source
# (FMA = 2, add / mul = 1, erfc / exp / rsqrt = 1 each).
P2P_FLOP_PER_UNORDERED_PAIR = 300.0

# HBM traffic of one P2P launch measured with rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE, calibrated against a copy of known size) for the kernel source
# with the recorded SHA-256; reported only while the source is unchanged.
P2P_COUNTERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "p2p_water_288000_counters.txt")
P2P_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2212_08284_amd", "csrc",
                          "ankh_p2p.hip")
FFT_COUNTERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "fft_cells_water_288000_counters.txt")
FFT_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2212_08284_amd", "csrc",
                          "ankh_fft.hip")

PEAK = {  # MI355X, TFLOP/s (hbm: GB/s)
    "hbm": 8000.0,
    "valu_fp64": 78.6,    # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
    "valu_fp32": 78.6,    # the same issue rate: packed FP32 (157.3) is not used by this build
    "valu_fp32_packed": 157.3,
    "mfma_fp64": 78.6,
    "mfma_fp32": 157.3,
    "mfma_bf16": 2500.0,
}


def p2p_traffic(counters=P2P_COUNTERS, source=P2P_SOURCE, leaves=None):
    """Calibrated HBM bytes per launch of a kernel from its committed counter summary, or None when
    the summary is missing, the kernel source has changed since, or it was taken on another leaf grid."""
    import hashlib
    try:
        rec = {}
        with open(counters) as fh:
            for ln in fh:
                if "=" in ln and not ln.lstrip().startswith("#"):
                    k, v = ln.split("=", 1)
                    rec[k.strip()] = v.strip()
        with open(source, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
        if rec.get("kernel_source_sha256") != sha:
            return None
        if leaves is not None and rec.get("leaves_per_axis") != str(leaves):
            return None
        return float(rec["fetch_bytes_per_launch"]) + float(rec["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def timed_run(plan, args_dev, steps, warmup, torch):
    """K timed steps with hipEvents around the M2L and pair-kernel stages only (every event idles the
    device for a few microseconds); then K more steps with an event at every stage boundary for the
    stage breakdown.  Returns (seconds per step, stats of the timed steps, breakdown, outputs)."""
    for _ in range(warmup):
        plan.energy_forces(*args_dev)
    torch.cuda.synchronize()
    plan.set_timing(2)
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = plan.energy_forces(*args_dev)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    stats = plan.get_stats()
    plan.set_timing(1)
    for _ in range(steps):
        plan.energy_forces(*args_dev)
    breakdown = plan.get_stats()["stage_ms"]
    plan.set_timing(0)
    plan.sync()
    return dt, stats, breakdown, out


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


def cpu_baseline(data, eps):
    """The classical-Ewald oracle on a bounded cut-out of the same water box."""
    import oracle
    import synth
    sub_edge = (2000 / synth.WATER_DENSITY) ** (1.0 / 3.0)     # ~2000 molecules, same density
    cut = synth.water_cutout(data, sub_edge)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = len(cut["q"])
    t0 = time.perf_counter()
    oracle.ewald(cut["pos"], cut["q"], cut["mu"], cut["theta"], edge=cut["edge"], eps=eps, nthreads=nthreads)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "atoms*evals/s", "cores": nthreads, "kind": "oracle",
            "sample": f"classical-Ewald oracle, energy+forces+fields, on a periodic cut-out of {n} atoms "
                      f"(whole molecules, edge {cut['edge']:.2f} A) of the benchmark box, accuracy {eps:g}; "
                      f"{dt:.2f} s wall; Ewald cost grows as N^1.5, so per-atom throughput at 288,000 atoms "
                      f"would be lower"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water_288000")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-only", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--mode", default="mixed_bf16x3", choices=["mixed", "mixed_bf16x3"],
                    help="precision mode of the headline (mixed) path")
    ap.add_argument("--no-induce", action="store_true", help="skip the induced-dipole solve")
    ap.add_argument("--no-derivs", action="store_true", help="skip the charge / quadrupole derivative timing")
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

    far_other = None
    if not args.no_far_compare:
        alt = "fft" if args.far == "fmm" else "fmm"
        pa = ak.Plan(n, rB, args.eps, 2, args.mode, far=alt, overlap=ovl, depth=args.depth)
        t_a, st_a, bd_a, out_a = timed_run(pa, args_dev, args.steps, args.warmup, torch)
        Em, Fm, Gm = [x.double().cpu().numpy() for x in out_mixed]
        Ea, Fa, Ga = [x.double().cpu().numpy() for x in out_a]
        far_other = {"far": alt, "ms_per_step": t_a * 1e3, "value": n / t_a, "plan_ms": st_a["plan_ms"],
                     "depth": st_a["depth"], "eq_order": st_a["eq_order"], "stage_ms": bd_a,
                     "rel_energy_diff": float(abs(Ea[0] - Em[0]) / abs(Em[0])),
                     "rel_rms_force_diff": rel_rms(Fa, Fm), "rel_rms_field_diff": rel_rms(Ga, Gm)}
        pa.close()
        log(f"{alt}: {far_other}")

    derivs = None
    if not args.no_derivs:
        derivs, dmix = derivs_run(pm, args_dev, torch)
        derivs["ms_energy_forces_fields"] = t_mixed * 1e3
        log(f"derivs: {derivs}")

    induce = None
    if not args.no_induce and args.workload.startswith("water"):
        induce = induce_run(pm, args_dev, synth.water_polarisabilities(n // 3), args.induce_tol, torch, dev)
        log(f"induce: { {k: v for k, v in induce.items() if k != '_mu'} }")

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
        Em, Fm, Gm = [x.double().cpu().numpy() for x in out_mixed]
        Ef, Ff, Gf = [x.double().cpu().numpy() for x in out_fp64]
        res = {
            "fp64_ms_per_step": t_fp64 * 1e3,
            "fp64_value": n / t_fp64,
            "speedup_mixed_vs_fp64": t_fp64 / t_mixed,
            "mixed_vs_fp64": {"rel_energy_err": float(abs(Em[0] - Ef[0]) / abs(Ef[0])),
                              "rel_rms_force_err": rel_rms(Fm, Ff), "rel_rms_field_err": rel_rms(Gm, Gf)},
            "fp64_stage_ms": bd_fp64,
        }
        pf.close()

    # roofline of the dominant kernel of the timed (mixed) path, from the live hipEvent stage timings
    sm = st_mixed["stage_ms"]
    unordered = st_mixed["near_pairs"] / 2.0
    p2p_flops = unordered * P2P_FLOP_PER_UNORDERED_PAIR
    p2p_tf = p2p_flops / (sm["p2p"] * 1e-3) / 1e12
    m2l_flops = st_mixed["m2l_flops"]
    m2l_tf = m2l_flops / (sm["m2l"] * 1e-3) / 1e12
    m2l_peak = PEAK["mfma_bf16"] if args.mode == "mixed_bf16x3" else PEAK["mfma_fp32"]
    p2p_alone_tf = p2p_flops / (bd_mixed["p2p"] * 1e-3) / 1e12
    p2p_roof = {"kernel": "p2p", "bound": "alu", "achieved": p2p_tf, "peak": PEAK["valu_fp32"],
                "unit": "TFLOP/s", "frac": p2p_tf / PEAK["valu_fp32"],
                "traffic": p2p_traffic(leaves=st_mixed["leaves_per_axis"]),
                "flop_per_launch": p2p_flops, "unordered_pairs": unordered,
                "flop_per_unordered_pair": P2P_FLOP_PER_UNORDERED_PAIR, "avg_launch_ms": sm["p2p"],
                "frac_of_packed_fp32_peak": p2p_tf / PEAK["valu_fp32_packed"],
                "alone_avg_launch_ms": bd_mixed["p2p"], "alone_achieved": p2p_alone_tf,
                "alone_frac": p2p_alone_tf / PEAK["valu_fp32"],
                "note": "peak = 256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz (unpacked FP32, as issued); in the timed "
                        "steps the far-field chain runs beside the pair kernel on a second stream and shares its "
                        "CUs, so avg_launch_ms is longer than the kernel alone (alone_*: the breakdown pass, one "
                        "stream)"}
    m2l_roof = {"kernel": "m2l", "bound": "mfma", "achieved": m2l_tf, "peak": m2l_peak, "unit": "TFLOP/s",
                "frac": m2l_tf / m2l_peak, "traffic": None, "flop_per_launch": m2l_flops, "avg_launch_ms": sm["m2l"],
                "note": "algorithmic flops per cell of level e: 2 * 189 * r_e^2 (r_e the kept rank of the compressed "
                        "operators, n_u if uncompressed) + 4 * n_u * r_e for the basis change; the BF16x3 split issues 3x "
                        "the contraction flops", "ranks": st_mixed.get("m2l_rank")}
    if args.far == "fft":
        # stage 4 of ANKH-FFT is the cell-transform kernel: per launch it reads and writes the half
        # spectrum (complex float64) and reads the real spectrum, 40 B per kept node frequency and leaf
        pa = 2 * st_mixed["eq_order"] - 1
        nf = pa * pa * (pa // 2 + 1)
        nleaf = st_mixed["leaves_per_axis"] ** 3
        fft_bytes = 40.0 * nf * nleaf
        fft_gbs = fft_bytes / (sm["m2l"] * 1e-3) / 1e9
        m2l_roof = {"kernel": "fft_cells", "bound": "hbm", "achieved": fft_gbs, "peak": PEAK["hbm"], "unit": "GB/s",
                    "frac": fft_gbs / PEAK["hbm"],
                    "traffic": p2p_traffic(FFT_COUNTERS, FFT_SOURCE, st_mixed["leaves_per_axis"]),
                    "bytes_per_launch": fft_bytes,
                    "alone_avg_launch_ms": bd_mixed["m2l"],
                    "alone_achieved": fft_bytes / (bd_mixed["m2l"] * 1e-3) / 1e9,
                    "alone_frac": fft_bytes / (bd_mixed["m2l"] * 1e-3) / 1e9 / PEAK["hbm"],
                    "avg_launch_ms": sm["m2l"],
                    "passes": 3 if st_mixed["fft_split"] else 1,
                    "note": f"ANKH-FFT cell transforms (stage 4): {nf} kept node frequencies x {nleaf} leaves, each "
                            "read and written once as complex float64 and multiplied by the real spectrum (float64): "
                            "the algorithmic bytes.  " + (
                                "On this grid the transforms run in three passes through HBM (each value read and "
                                "written once per pass)" if st_mixed["fft_split"] else
                                "On this grid all cells of a node frequency sit in one block's LDS (one pass)") +
                            "; traffic is the counters' sum over the stage's launches"}
    roof, other = (p2p_roof, m2l_roof) if sm["p2p"] >= sm["m2l"] else (m2l_roof, p2p_roof)

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
        "dtype": "f32" if args.mode == "mixed" else "f32+bf16x3",
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
                         "stages in sequence on one stream; the timed steps overlap the far-field chain with the pair "
                         "kernel and carry events around stage 4 (the M2L, or the cell transforms of ANKH-FFT) and the "
                         "pair kernel only.  ANKH-FFT stages: m2m = forward node transform, m2l = cell transforms "
                         "with the spectrum, l2l = inverse node transform + leaf energies, periodic = none",
        "roofline": roof,
        "roofline_" + other["kernel"]: other,
    }
    line.update(res)
    if far_other is not None:
        line["far_other"] = far_other
    if derivs is not None:
        line["derivs"] = derivs
    if induce is not None:
        induce.pop("_mu", None)
        line["induce"] = induce
    pm.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(data, args.eps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Writes the stored expected values of the parity tests.

Calls only the seeded generators (synth) and the classical-Ewald oracle
(oracle/); nothing here touches the GPU library.  Run from the repository
root:  python tests/golden/make_golden.py [name ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

EPS = 1e-11


def make(name):
    out = os.path.join(HERE, f"{name}.npz")
    t = time.time()
    if name == "charges_1000":
        d = synth.workload(name)
        r = oracle.ewald(d["pos"], d["q"], edge=d["edge"], eps=EPS, grad=True)
        np.savez_compressed(out, energy=r["energy"], forces=r["forces"], eps=EPS)
    elif name == "water_9000":
        d = synth.workload(name)
        r = oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=d["edge"], eps=EPS, grad=True)
        np.savez_compressed(out, energy=r["energy"], forces=r["forces"], dEdmu=r["dEdmu"], eps=EPS)
    elif name == "water_288000_sites":
        # forces and fields on 32 seeded atoms of the 288,000-atom box, one by one
        d = synth.workload("water_288000")
        sel = np.sort(np.random.default_rng(33).choice(len(d["q"]), 32, replace=False))
        r = oracle.ewald_sites(d["pos"], d["q"], d["mu"], d["theta"], d["edge"], sel, eps=1e-9,
                               alpha=0.1)
        np.savez_compressed(out, sel=sel, forces=r["forces"], dEdmu=r["dEdmu"], eps=1e-9)
    elif name == "ionic_1000000_sites":
        # forces and fields on 32 seeded ions of the 1,000,000-ion melt (charges + dipoles), one by one
        d = synth.workload("ionic_1000000")
        sel = np.sort(np.random.default_rng(44).choice(len(d["q"]), 32, replace=False))
        r = oracle.ewald_sites(d["pos"], d["q"], d["mu"], d["theta"], d["edge"], sel, eps=1e-9,
                               alpha=0.05)
        np.savez_compressed(out, sel=sel, forces=r["forces"], dEdmu=r["dEdmu"], eps=1e-9)
    elif name == "water_cutout_20k":
        # the whole classical-Ewald solution on the corner cut-out (58.442 A) of the 3,000,000-molecule box
        d = synth.water_cutout(synth.workload("water_9000000"), 58.442)
        r = oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=d["edge"], eps=1e-10, grad=True)
        np.savez_compressed(out, energy=r["energy"], forces=r["forces"], dEdmu=r["dEdmu"], n=len(d["q"]),
                            eps=1e-10)
    elif name == "water_288000_energy":
        d = synth.workload("water_288000")
        r = oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=d["edge"], eps=1e-9, grad=False)
        np.savez_compressed(out, energy=r["energy"], e_real=r["e_real"], e_rec=r["e_rec"],
                            e_self=r["e_self"], e_bg=r["e_bg"], eps=1e-9)
    elif name == "ionic_1000000_energy":
        d = synth.workload("ionic_1000000")
        r = oracle.ewald(d["pos"], d["q"], d["mu"], d["theta"], edge=d["edge"], eps=1e-9, grad=False)
        np.savez_compressed(out, energy=r["energy"], e_real=r["e_real"], e_rec=r["e_rec"],
                            e_self=r["e_self"], e_bg=r["e_bg"], eps=1e-9)
    else:
        raise KeyError(name)
    print(f"{name}: {time.time() - t:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["charges_1000", "water_9000", "water_288000_sites"]
    for nm in names:
        make(nm)

"""Write full-size expected values of the DF-DSRG-PT2 pass with the FP64 oracle.

Only ``synth`` (seeded inputs) and ``oracle`` are used; nothing here touches
the HIP path.  Output: ``tests/golden/<config>_s<s>.json`` with the energy
(double-double), the occupation numbers, the diagonal of D_vv, its trace,
per-pair energies of a few sampled pairs, and for every p_o of the workload the
kept count, its margins, the kept-space energy and the correction.

Usage: python tests/golden/make_golden.py c2 [c3 ...]   (c3: ~5 min per s on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dsrg_pt2 as o  # noqa: E402


def sampled_pairs(n_core, k=6, seed=0):
    rng = np.random.default_rng(seed)
    pairs = {(0, 0), (0, max(0, n_core - 1)), (n_core - 1, n_core - 1)}
    while len(pairs) < min(k, n_core * (n_core + 1) // 2):
        i, j = sorted(rng.integers(0, n_core, 2))
        pairs.add((int(i), int(j)))
    return sorted(pairs)


def make(name: str, s: float):
    cfg = synth.CONFIGS[name]
    t0 = time.time()
    inp = synth.config_inputs(name)
    r = o.pt2_pass_inputs(inp, s)
    t_pass = time.time() - t0
    occ, vecs = o.natural_orbitals(r.D_vv)
    out = dict(config=name, sizes=list(cfg["sizes"]), seed=0, s=s,
               energy=list(r.energy), trace=float(np.trace(r.D_vv)),
               D_diag=np.diag(r.D_vv).tolist(), occ=occ.tolist(),
               pairs=[], truncation=[], oracle_seconds=dict(pass_=t_pass))
    if inp.n_core:
        for i, j in sampled_pairs(inp.n_core):
            out["pairs"].append(dict(i=i, j=j, energy=float(r.pair_energy[i, j]),
                                     tnorm=float(r.pair_tnorm[i, j])))
    for p_o in cfg["p_o"]:
        n_kept, margins = o.kept_count_po(occ, p_o)
        t1 = time.time()
        e_kept = o.kept_energy(inp, vecs, n_kept, s)
        out["truncation"].append(dict(p_o=p_o, n_kept=n_kept, margins=list(margins),
                                      e_kept=list(e_kept),
                                      correction=list(o.pt2_correction(r.energy, e_kept)),
                                      kept_seconds=time.time() - t1))
    path = os.path.join(HERE, f"{name}_s{s:g}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{path}: E={r.energy[0]:.10f} kept={[t['n_kept'] for t in out['truncation']]} "
          f"({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["c2"]:
        for s in synth.CONFIGS[name]["s"]:
            make(name, s)

"""The headline workload's sizes at full size (80 core holes, 1200 virtuals, 4000
auxiliary functions, p_o = 0.985) at both flow parameters of the workload,
s = 0.5 and 1.0 Eh^-2, in the launch configuration bench.py times, against the
FP64 oracle's expected values (tests/golden/c3_s0.5.json and c3_s1.json, written
by make_golden.py from the oracle alone): the energy, six sampled pair
energies, the diagonal of D_vv, every occupation number, the kept count and the
correction.  Three paths: FP64 (1e-8 Eh), split BF16 with four slices for both
products (the default mixed path, 1e-6 Eh) and INT8 digits (1e-6 Eh).  The
correction bound is max(tol, 2e-15 |E_kept|): the natural orbitals of two FP64
eigensolvers agree only to rounding (see test_gpu_c5.py).  About half a minute per s."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from gpu_common import dd_diff, need_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("golden", ["c3_s0.5.json", "c3_s1.json"])
def test_c3_full_size_against_golden(golden):
    dp = need_gpu()
    with open(os.path.join(HERE, "golden", golden)) as f:
        gold = json.load(f)
    s = float(gold["s"])
    assert tuple(gold["sizes"]) == (80, 0, 1200, 4000)
    tr = gold["truncation"][0]
    occ_ref = np.array(gold["occ"])
    diag_ref = np.array(gold["D_diag"])
    print(f"c3: drawing inputs (s = {s})", flush=True)
    inp = synth.config_inputs("c3")
    d = dp.upload_inputs(inp)
    del inp
    e_kept = abs(sum(tr["e_kept"]))
    for precision, tol, rel in ((dp.FP64, 1e-8, 1e-11), (dp.BF16_SLICED, 1e-6, 1e-9), (dp.INT8_SLICED, 1e-6, 1e-9)):
        print(f"c3: precision {precision}", flush=True)
        opts = dp.make_opts(80, 0, 1200, 4000, s, precision=precision)
        r = dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], want_pair_energy=True)
        e = r["e_pt2"].cpu().numpy()
        dE = dd_diff((float(e[0]), float(e[1])), gold["energy"])
        pe = r["pair_energy"].cpu().numpy()
        dpair = max(abs(pe[q["i"], q["j"]] - q["energy"]) for q in gold["pairs"])
        ddiag = np.abs(np.diag(r["D_vv"].cpu().numpy()) - diag_ref).max()
        t = dp.fno_truncate(r["D_vv"], tr["p_o"])
        occ = t["occ"].cpu().numpy()
        # kept-space energy in the build's precision, and (after BF16) in INT8 digits as the benchmark runs it
        dC = 0.0
        for cp in ((precision, dp.INT8_SLICED) if precision == dp.BF16_SLICED else (precision,)):
            oc = dp.make_opts(80, 0, 1200, 4000, s, precision=cp)
            c = dp.pt2_energy_correction(oc, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], t["no_vecs"],
                                         t["n_kept"], r["e_pt2"])
            cc = c["correction"].cpu().numpy()
            dC = max(dC, dd_diff((float(cc[0]), float(cc[1])), tr["correction"]))
        dON = np.abs(occ - occ_ref).max()
        print(f"  dE {dE:.3e} Eh, max dE_pair {dpair:.3e}, max dD_aa {ddiag:.3e}, kept {t['n_kept']} "
              f"(oracle {tr['n_kept']}), dcorr {dC:.3e} Eh, max dON {dON:.3e}", flush=True)
        assert dE <= tol
        assert dpair <= tol
        assert ddiag <= rel * diag_ref.max()
        assert dON <= rel * occ_ref.max()
        assert t["n_kept"] == tr["n_kept"]
        assert dC <= max(tol, 2e-15 * e_kept)
        del r, t, c
        torch.cuda.empty_cache()

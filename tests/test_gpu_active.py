"""GPU parity of the active-hole path (row a6): Eq. A9's S(.) and Gamma^{uv}_{xy}
terms through the natural-orbital rotation of Gamma_act, against the literal
FP64 oracle contraction."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from gpu_common import dd_diff, gpu_pass, need_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [
    ("small", (3, 2, 70, 50), 0.5, None),
    ("ragged", (5, 4, 131, 77), 0.7, None),
    ("no_core", (0, 4, 64, 40), 0.5, None),
    ("full_occ", (3, 2, 66, 30), 0.5, "two"),
    ("empty_occ", (3, 2, 66, 30), 0.5, "zero"),
    ("one_active", (2, 2, 70, 45), 0.9, "diag"),
    # the core-active rotation kernel keeps up to 8 / 16 / 32 active matrices per
    # thread; beyond 32 the rotation runs as an FP64 GEMM
    ("act10", (2, 10, 70, 40), 0.6, None),
    ("act18", (1, 18, 65, 36), 0.5, None),
    ("act34", (1, 34, 34, 16), 0.5, None),
]


_REF = {}  # oracle results per case, shared by the two precisions


@pytest.mark.parametrize("name,sizes,s,gmod", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "bf16"])
def test_active_pass_parity(name, sizes, s, gmod, precision):
    inp = synth.generate(*sizes, seed=4)
    if gmod == "two":
        inp = inp.replace(gamma_act=2.0 * np.eye(inp.n_act))
    elif gmod == "zero":
        inp = inp.replace(gamma_act=np.zeros((inp.n_act, inp.n_act)))
    elif gmod == "diag":
        inp = inp.replace(gamma_act=np.diag([1.7, 0.3]))
    print(f"case {name} sizes={sizes} precision={precision}", flush=True)
    if name not in _REF:
        _REF[name] = o.pt2_pass_inputs(inp, s)
    ref = _REF[name]
    g = gpu_pass(inp, s, precision=precision)
    tol_e = 1e-8 if precision == 0 else 1e-6
    assert dd_diff(g["energy"], ref.energy) <= max(tol_e, 1e-12 * abs(ref.E))
    scale = max(np.abs(ref.D_vv).max(), 1e-300)
    assert np.abs(g["D"] - ref.D_vv).max() <= (1e-11 if precision == 0 else 1e-8) * scale
    assert np.array_equal(g["D"], g["D"].T)
    act = np.isnan(ref.pair_energy)
    assert np.all(np.isnan(g["pair_energy"][act]))
    np.testing.assert_allclose(g["pair_energy"][~act], ref.pair_energy[~act], rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(g["pair_tnorm"], ref.pair_tnorm, rtol=1e-6, atol=1e-30)


def test_c2_full_size_against_golden():
    """c2 (40 core, 8 active, 400 virtuals, 1600 aux, rank-64 B): energy, every
    occupation number, kept counts at the three p_o and the corrections."""
    dp = need_gpu()
    with open(os.path.join(HERE, "golden", "c2_s0.5.json")) as f:
        gold = json.load(f)
    inp = synth.config_inputs("c2")
    g = gpu_pass(inp, 0.5)
    assert dd_diff(g["energy"], gold["energy"]) <= 1e-8
    occ_ref = np.array(gold["occ"])
    for tr in gold["truncation"]:
        t = dp.fno_truncate(g["raw"]["D_vv"], tr["p_o"])
        occ = t["occ"].cpu().numpy()
        assert np.abs(occ - occ_ref).max() <= 1e-11 * occ_ref.max()
        assert t["n_kept"] == tr["n_kept"]
        d = g["dev"]
        c = dp.pt2_energy_correction(g["opts"], d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"],
                                     t["no_vecs"], t["n_kept"], g["raw"]["e_pt2"])
        cc = c["correction"].cpu().numpy()
        assert dd_diff((cc[0], cc[1]), tr["correction"]) <= 1e-8


@pytest.mark.parametrize("precision,name", [(1, "bf16"), (3, "int8")])
def test_c2_mixed_against_golden(precision, name):
    """c2 through the mixed paths (split BF16, INT8 digits): the active blocks
    store amplitudes while the core pairs of the kept-space energy run through
    the energy-only product; energy, occupation numbers, kept counts at the
    three p_o and the corrections against the oracle's values at the mixed bound
    (1e-6 Eh)."""
    dp = need_gpu()
    with open(os.path.join(HERE, "golden", "c2_s0.5.json")) as f:
        gold = json.load(f)
    inp = synth.config_inputs("c2")
    g = gpu_pass(inp, 0.5, precision=precision)
    dE = dd_diff(g["energy"], gold["energy"])
    occ_ref = np.array(gold["occ"])
    for tr in gold["truncation"]:
        t = dp.fno_truncate(g["raw"]["D_vv"], tr["p_o"])
        occ = t["occ"].cpu().numpy()
        d = g["dev"]
        c = dp.pt2_energy_correction(g["opts"], d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"],
                                     t["no_vecs"], t["n_kept"], g["raw"]["e_pt2"])
        cc = c["correction"].cpu().numpy()
        dC = dd_diff((cc[0], cc[1]), tr["correction"])
        print(f"c2 {name} p_o {tr['p_o']}: dE {dE:.3e}, max dON {np.abs(occ - occ_ref).max():.3e}, "
              f"kept {t['n_kept']} ({tr['n_kept']}), dcorr {dC:.3e}", flush=True)
        assert np.abs(occ - occ_ref).max() <= 1e-9 * occ_ref.max()
        assert t["n_kept"] == tr["n_kept"]
        assert dC <= 1e-6
    assert dE <= 1e-6

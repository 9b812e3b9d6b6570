"""GPU parity of the split-FP8 path (e4m3 slices, per-block E8M0 scales, scaled
MFMA with FP32 accumulation) against the FP64 oracle, through the C ABI.

Bound derived from the arithmetic: each 32-wide block of a row of B is carried by
NS slices to within half a unit of the last one, 2^(E - 4 - 5(NS-1) - 1) <=
m 2^-(5 NS - 1) with m the block's largest magnitude; the products of two rows, the
dropped slice levels and the FP32 accumulation (relative 2^-24 per step) stay below
a few times that, relative to the product of the row norms.  The energy is
quadratic in V and D is quadratic in T, so the tests allow 8 x 2^-(5 NS - 1)
relative to |E| and to max|D| (1.5e-5 at NS = 4).  This path does not reach the
1e-6 Eh target of the mixed path beyond small systems; the BF16 path does.
"""
import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from gpu_common import dd_diff, gpu_pass, need_gpu

pytestmark = pytest.mark.gpu

FP8 = 2


def bound(ns):
    return 8.0 * 2.0 ** -(5 * ns - 1)


CASES = [
    ("c1", None, 0.5),
    ("ragged_odd", (7, 0, 131, 77), 0.5),
    ("tiles_ragged", (12, 0, 200, 256), 1.0),
    ("one_hole", (1, 0, 70, 33), 0.8),
    ("active", (6, 4, 90, 140), 0.5),
]


@pytest.mark.parametrize("name,sizes,s", CASES, ids=[c[0] for c in CASES])
def test_fp8_pass_parity(name, sizes, s):
    inp = synth.config_inputs("c1") if sizes is None else synth.generate(*sizes, seed=3)
    print(f"case {name} sizes={sizes} s={s}", flush=True)
    ref = o.pt2_pass_inputs(inp, s)
    g = gpu_pass(inp, s, precision=FP8)
    dE = dd_diff(g["energy"], ref.energy)
    print(f"  dE {dE:.3e} Eh (rel {dE / abs(ref.E):.2e})", flush=True)
    assert dE <= bound(4) * abs(ref.E)
    scale = np.abs(ref.D_vv).max()
    assert np.abs(g["D"] - ref.D_vv).max() <= bound(4) * scale
    assert np.array_equal(g["D"], g["D"].T)
    ok = np.isfinite(ref.pair_energy)
    np.testing.assert_allclose(g["pair_energy"][ok], ref.pair_energy[ok], rtol=bound(4),
                               atol=bound(4) * np.abs(ref.pair_energy[ok]).max())


def test_fp8_error_falls_with_slices():
    inp = synth.generate(12, 0, 200, 256, seed=3)
    ref = o.pt2_pass_inputs(inp, 1.0)
    errs = []
    for ns in (2, 3, 4):
        g = gpu_pass(inp, 1.0, precision=FP8, slices_gemm1=ns)
        errs.append(dd_diff(g["energy"], ref.energy) / abs(ref.E))
    print("relative energy errors by FP8 slice count:", errs, flush=True)
    assert errs[0] > errs[1] > errs[2]
    for ns, e in zip((2, 3, 4), errs):
        assert e <= bound(ns)


def test_fp8_localized_blocks():
    """Per-block scales: rows whose magnitudes decay along the auxiliary index."""
    inp = synth.generate(10, 0, 150, 300, seed=4, localized_xi=1.0)
    ref = o.pt2_pass_inputs(inp, 0.5)
    g = gpu_pass(inp, 0.5, precision=FP8)
    assert dd_diff(g["energy"], ref.energy) <= bound(4) * abs(ref.E)
    assert np.abs(g["D"] - ref.D_vv).max() <= bound(4) * np.abs(ref.D_vv).max()


def test_fp8_truncation_and_correction_c1():
    dp = need_gpu()
    inp = synth.config_inputs("c1")
    ref = o.full_pipeline(inp, 0.5, 0.985)
    g = gpu_pass(inp, 0.5, precision=FP8)
    t = dp.fno_truncate(g["raw"]["D_vv"], 0.985)
    assert t["n_kept"] == ref["n_kept"]
    occ = t["occ"].cpu().numpy()
    assert np.abs(occ - ref["occ"]).max() <= bound(4) * ref["occ"].max()
    d = g["dev"]
    c = dp.pt2_energy_correction(g["opts"], d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], t["no_vecs"],
                                 t["n_kept"], g["raw"]["e_pt2"])
    cc = c["correction"].cpu().numpy()
    assert dd_diff((cc[0], cc[1]), ref["correction"]) <= bound(4) * abs(sum(ref["energy"]))

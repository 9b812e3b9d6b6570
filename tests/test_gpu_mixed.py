"""GPU parity of the split-BF16 path against the FP64 oracle (through the C ABI).

Bar for the mixed path: energy within 1e-6 Eh, kept counts exact, and the error
shrinking as slices are added (the slicing error is 2^-(8 + 9(k-1)) relative).
"""
import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from gpu_common import dd_diff, gpu_pass, need_gpu

pytestmark = pytest.mark.gpu

BF16 = 1
E_TOL_MIXED = 1e-6

CASES = [
    ("c1", None, 0.5),
    ("ragged_odd", (7, 0, 131, 77), 0.5),
    ("tiles_ragged", (12, 0, 200, 256), 1.0),
    ("one_hole", (1, 0, 70, 33), 0.8),
    # one hole, three 128-row tile rows: every pair is i == j, whose V^{ii} the product
    # kernel computes only on and above the diagonal (the epilogue takes Q from P)
    ("one_hole_tiles", (1, 0, 300, 96), 0.5),
    # n_v a multiple of the 128-row tile (no padding rows or columns anywhere) and an
    # auxiliary count that is a whole number of contraction chunks
    ("aligned", (6, 0, 256, 128), 0.5),
]


@pytest.mark.parametrize("name,sizes,s", CASES, ids=[c[0] for c in CASES])
def test_bf16_pass_parity(name, sizes, s):
    inp = synth.config_inputs("c1") if sizes is None else synth.generate(*sizes, seed=3)
    print(f"case {name} sizes={sizes} s={s}", flush=True)
    ref = o.pt2_pass_inputs(inp, s)
    g = gpu_pass(inp, s, precision=BF16)
    dE = dd_diff(g["energy"], ref.energy)
    assert dE <= E_TOL_MIXED
    assert dE <= 1e-9 * abs(ref.E)          # ~ 2^-34 relative slicing error, with margin
    scale = np.abs(ref.D_vv).max()
    assert np.abs(g["D"] - ref.D_vv).max() <= 1e-8 * scale
    assert np.array_equal(g["D"], g["D"].T)
    ok = np.isfinite(ref.pair_energy)
    np.testing.assert_allclose(g["pair_energy"][ok], ref.pair_energy[ok], rtol=1e-8, atol=1e-12)


def test_bf16_error_falls_with_slices():
    inp = synth.generate(6, 0, 96, 130, seed=11)
    ref = o.pt2_pass_inputs(inp, 0.5)
    errs = []
    for ns in (2, 3, 4):
        g = gpu_pass(inp, 0.5, precision=BF16, slices_gemm1=ns)
        errs.append(dd_diff(g["energy"], ref.energy) / abs(ref.E))
    print("relative energy errors by slice count:", errs, flush=True)
    # with the exact FP64 diagonal of V^{ii} the remaining error is the zero-mean
    # dropped level; NumPy emulation of the same slicing gives 1.4e-7, 7.2e-11, 3.1e-13
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 1e-6 and errs[1] < 1e-9 and errs[2] < 3e-12


def test_bf16_truncation_and_correction_c1():
    dp = need_gpu()
    inp = synth.config_inputs("c1")
    ref = o.full_pipeline(inp, 0.5, 0.985)
    g = gpu_pass(inp, 0.5, precision=BF16)
    t = dp.fno_truncate(g["raw"]["D_vv"], 0.985)
    assert t["n_kept"] == ref["n_kept"]
    d = g["dev"]
    c = dp.pt2_energy_correction(g["opts"], d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], t["no_vecs"],
                                 t["n_kept"], g["raw"]["e_pt2"])
    cc = c["correction"].cpu().numpy()
    assert dd_diff((cc[0], cc[1]), ref["correction"]) <= E_TOL_MIXED


def test_bf16_density_slices():
    """Split-BF16 density product (default, 4 slices) against the FP64 density kernel
    on the same BF16 amplitudes and against the oracle; the error of D falls with the
    density slice count (about 2^-(9k-1) relative for k slices)."""
    inp = synth.generate(9, 0, 150, 200, seed=5)
    ref = o.pt2_pass_inputs(inp, 0.5)
    scale = np.abs(ref.D_vv).max()
    g64 = gpu_pass(inp, 0.5, precision=BF16, slices_gemm2=1)
    errs = []
    e_split = None
    for k in (2, 3, 4):
        g = gpu_pass(inp, 0.5, precision=BF16, slices_gemm2=k)
        # the energy does not involve the density product: bitwise the same for every
        # slice count; against the FP64-density pass (whose epilogue stores FP64
        # amplitudes and sums each tile's energy terms in another order) up to rounding
        e_split = e_split or g["energy"]
        assert g["energy"] == e_split
        assert dd_diff(g["energy"], g64["energy"]) <= 1e-14 * abs(g64["energy"][0])
        assert np.array_equal(g["D"], g["D"].T)
        errs.append(np.abs(g["D"] - ref.D_vv).max() / scale)
    print("relative D errors by density slice count:", errs,
          "FP64 density:", np.abs(g64["D"] - ref.D_vv).max() / scale, flush=True)
    assert errs[0] > errs[1] > errs[2]
    for k, e in zip((2, 3, 4), errs):
        assert e <= 16.0 * 2.0 ** -(9 * k - 1) + 1e-11
    assert np.abs(g["D"] - g64["D"]).max() <= 1e-10 * scale


def test_bf16_density_reproducible_and_batched():
    """Fixed-order split reduction: repeated runs are bitwise equal, and batching the
    pairs differently changes D only at the rounding level."""
    inp = synth.generate(11, 0, 130, 96, seed=8)
    a = gpu_pass(inp, 0.5, precision=BF16)
    b = gpu_pass(inp, 0.5, precision=BF16)
    assert np.array_equal(a["D"], b["D"]) and a["energy"] == b["energy"]
    c = gpu_pass(inp, 0.5, precision=BF16, pair_batch=7)
    assert np.abs(c["D"] - a["D"]).max() <= 1e-12 * np.abs(a["D"]).max()


def test_bf16_range_guard():
    """A row of B whose largest magnitude lies below the range BF16 slicing keeps
    exact (2^(E_min - 1), E_min = 8 - (126 - 9 (k - 1)) // 2 = -41 at k = 4 slices)
    makes the BF16 pass return DFPT2_ERR_UNSUPPORTED instead of losing the bits
    silently; FP64 and INT8 digits accept the same input, and a row just inside
    the range passes the guard and stays at parity with the oracle."""
    dp = need_gpu()
    from paper_2312_07008_amd._lib import ERR_UNSUPPORTED, DfptError
    inp = synth.generate(4, 0, 40, 64, seed=11)
    m = np.abs(inp.B[1, 7]).max()
    tiny = inp.B.copy()
    tiny[1, 7] *= 2.0 ** -60 / m                     # max |row| = 2^-60 < 2^-42
    inside = inp.B.copy()
    inside[1, 7] *= 2.0 ** -41.5 / m                 # frexp exponent -41 = E_min
    t = inp.replace(B=tiny)
    print("range guard: BF16 with a row at 2^-60", flush=True)
    with pytest.raises(DfptError) as ex:
        gpu_pass(t, 0.5, precision=BF16)
    assert ex.value.status == ERR_UNSUPPORTED
    print(f"  status {ex.value.status}: {ex.value}", flush=True)
    ref = o.pt2_pass_inputs(t, 0.5)
    for prec, tol in ((dp.FP64, 1e-12), (dp.INT8_SLICED, 1e-9)):
        g = gpu_pass(t, 0.5, precision=prec)
        assert dd_diff(g["energy"], ref.energy) <= tol * abs(ref.E)
    ok = inp.replace(B=inside)
    g = gpu_pass(ok, 0.5, precision=BF16)
    ref = o.pt2_pass_inputs(ok, 0.5)
    assert dd_diff(g["energy"], ref.energy) <= 1e-9 * abs(ref.E)

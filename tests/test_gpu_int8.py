"""GPU parity of the INT8-digit path (balanced base-256 digits per row, exact INT32
level sums on the INT8 MFMA, for V = B B^T and for the density product) against the
FP64 oracle, through the C ABI.

Bar derived from the arithmetic: with k digits every row is represented to within
2^-(7 + 8(k-1)) of its largest element, the level sums are exact, and the levels
>= k that the kernel drops are below 2^-(8k - 2) of the product of the row scales.
A NumPy emulation of the same digits (exact integer sums, FP64 diagonal of V^{ii})
gives relative energy errors 3.5e-8, 3.7e-11, 3.6e-13 at k = 3, 4, 5 on the
`falls_with_digits` input; the GPU sums the same integers, so it must land on the
same values up to FP64 rounding of the epilogue.
"""
import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from gpu_common import dd_diff, gpu_pass, need_gpu

pytestmark = pytest.mark.gpu

INT8 = 3
E_TOL_MIXED = 1e-6

CASES = [
    ("c1", None, 0.5),
    ("ragged_odd", (7, 0, 131, 77), 0.5),
    ("tiles_ragged", (12, 0, 200, 256), 1.0),
    ("one_hole", (1, 0, 70, 33), 0.8),
    # one hole, three 128-row tile rows: every pair is i == j, whose V^{ii} the product
    # kernel forms only on and above the diagonal (the epilogue takes Q from P)
    ("one_hole_tiles", (1, 0, 300, 96), 0.5),
    ("active", (6, 4, 90, 140), 0.5),
    # n_v a multiple of the 128-row tile (no padding rows or columns anywhere) and an
    # auxiliary count that is a whole number of contraction chunks
    ("aligned", (6, 0, 256, 128), 0.5),
]


@pytest.mark.parametrize("name,sizes,s", CASES, ids=[c[0] for c in CASES])
def test_int8_pass_parity(name, sizes, s):
    inp = synth.config_inputs("c1") if sizes is None else synth.generate(*sizes, seed=3)
    print(f"case {name} sizes={sizes} s={s}", flush=True)
    ref = o.pt2_pass_inputs(inp, s)
    g = gpu_pass(inp, s, precision=INT8)
    dE = dd_diff(g["energy"], ref.energy)
    print(f"  dE {dE:.3e} Eh (rel {dE / abs(ref.E):.2e})", flush=True)
    assert dE <= E_TOL_MIXED
    assert dE <= 1e-9 * abs(ref.E)
    scale = np.abs(ref.D_vv).max()
    assert np.abs(g["D"] - ref.D_vv).max() <= 1e-8 * scale
    assert np.array_equal(g["D"], g["D"].T)
    ok = np.isfinite(ref.pair_energy)
    np.testing.assert_allclose(g["pair_energy"][ok], ref.pair_energy[ok], rtol=1e-8, atol=1e-12)


def test_int8_error_falls_with_digits():
    inp = synth.generate(6, 0, 96, 130, seed=11)
    ref = o.pt2_pass_inputs(inp, 0.5)
    errs = []
    for k in (3, 4, 5):
        g = gpu_pass(inp, 0.5, precision=INT8, slices_gemm1=k, slices_gemm2=1)
        errs.append(dd_diff(g["energy"], ref.energy) / abs(ref.E))
    print("relative energy errors by digit count:", errs, flush=True)
    emulated = (3.492777855885096e-08, 3.680530242592002e-11, 3.627844019530811e-13)
    assert errs[0] > errs[1] > errs[2]
    for e, em in zip(errs, emulated):
        assert abs(e - em) <= 0.05 * em + 1e-15


@pytest.mark.parametrize("span,slices_gemm2", [(60, 1), (20, 0)])
def test_int8_wide_row_scales(span, slices_gemm2):
    """Rows whose magnitudes span 2^-span .. 2^span: digits carry no exponent, so every
    row keeps its full precision relative to its own scale.  At span 60 the density
    runs in FP64 (slices_gemm2 = 1): the BF16 density slices are true-scale and their
    products accumulate in FP32, whose range (2^128) amplitudes of 2^100 would exceed."""
    inp = synth.generate(5, 0, 100, 96, seed=8)
    rng = np.random.default_rng(1)
    k = rng.integers(-span, span + 1, size=(inp.n_h, inp.n_vir))
    inp = inp.replace(B=inp.B * np.ldexp(1.0, k)[:, :, None])
    ref = o.pt2_pass_inputs(inp, 0.5)
    g = gpu_pass(inp, 0.5, precision=INT8, slices_gemm2=slices_gemm2)
    assert dd_diff(g["energy"], ref.energy) <= 1e-9 * abs(ref.E)
    assert np.abs(g["D"] - ref.D_vv).max() <= 1e-8 * np.abs(ref.D_vv).max()


def test_int8_pass_is_reproducible():
    """Two runs are bitwise equal (fixed reduction orders, exact integer sums)."""
    inp = synth.generate(9, 0, 150, 200, seed=5)
    ref = o.pt2_pass_inputs(inp, 0.5)
    g1 = gpu_pass(inp, 0.5, precision=INT8)
    g2 = gpu_pass(inp, 0.5, precision=INT8)
    assert np.array_equal(g1["D"], g2["D"])
    assert g1["energy"] == g2["energy"]
    assert np.abs(g1["D"] - ref.D_vv).max() <= 1e-8 * np.abs(ref.D_vv).max()


def test_int8_truncation_and_correction_c1():
    dp = need_gpu()
    inp = synth.config_inputs("c1")
    ref = o.full_pipeline(inp, 0.5, 0.985)
    g = gpu_pass(inp, 0.5, precision=INT8)
    t = dp.fno_truncate(g["raw"]["D_vv"], 0.985)
    assert t["n_kept"] == ref["n_kept"]
    d = g["dev"]
    c = dp.pt2_energy_correction(g["opts"], d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], t["no_vecs"],
                                 t["n_kept"], g["raw"]["e_pt2"])
    cc = c["correction"].cpu().numpy()
    assert dd_diff((cc[0], cc[1]), ref["correction"]) <= E_TOL_MIXED


def test_int8_density_digits():
    """INT8-digit density (default 5 digits) against the FP64 density kernel on the same
    amplitudes and against the oracle; its error falls with the digit count.  NumPy
    emulation of the same digits on this input: 1.3e-4, 7.9e-7, 3.3e-9 of max|D| at
    2, 3, 4 digits (off-diagonal; the diagonal is the exact FP64 sum)."""
    inp = synth.generate(9, 0, 150, 200, seed=5)
    ref = o.pt2_pass_inputs(inp, 0.5)
    scale = np.abs(ref.D_vv).max()
    g64 = gpu_pass(inp, 0.5, precision=INT8, slices_gemm2=1)
    errs = []
    for k in (2, 3, 4, 5):
        g = gpu_pass(inp, 0.5, precision=INT8, slices_gemm2=k)
        errs.append(np.abs(g["D"] - g64["D"]).max() / scale)
        assert np.array_equal(g["D"], g["D"].T)
        assert g["energy"] == g64["energy"]      # the density does not touch the energy
    print("relative D errors by density digit count:", errs, flush=True)
    emulated = (1.2877e-4, 7.9016e-7, 3.2780e-9)
    for e, em in zip(errs, emulated):
        assert e <= 2.0 * em
    assert errs[0] > errs[1] > errs[2] > errs[3]
    g = gpu_pass(inp, 0.5, precision=INT8)
    assert np.abs(g["D"] - ref.D_vv).max() <= 1e-8 * scale

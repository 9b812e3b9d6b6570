"""Pins of the NAF oracle (oracle/naf.py) against facts that do not come from it."""
import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from oracle import naf


def test_all_functions_kept_is_exact():
    """eps <= 0 keeps every NAF: U is orthogonal, so V = B B^T and the whole pass
    (energy and D) are unchanged."""
    inp = synth.generate(5, 2, 40, 60, seed=4)
    Bt, sigma, n = naf.naf_compress(inp.B, 0.0)
    assert n == inp.n_aux
    a = o.pt2_pass_inputs(inp, 0.5)
    b = o.pt2_pass_inputs(inp.replace(B=Bt), 0.5)
    assert abs(a.E - b.E) <= 1e-12 * abs(a.E)
    assert np.abs(a.D_vv - b.D_vv).max() <= 1e-12 * np.abs(a.D_vv).max()


def test_dropped_norm_equals_dropped_eigenvalues():
    """sum ||B||^2 - sum ||B~||^2 = sum of the dropped sigma (trace of W)."""
    inp = synth.generate(4, 0, 30, 50, seed=1, localized_xi=2.0)
    sigma_all = naf.naf_compress(inp.B, 0.0)[1]
    eps = float(sigma_all[20] / sigma_all[0])   # keeps exactly 20 functions (no ties)
    Bt, sigma, n = naf.naf_compress(inp.B, eps)
    assert n == 20
    dropped = np.sum(inp.B ** 2) - np.sum(Bt ** 2)
    assert abs(dropped - sigma[20:].sum()) <= 1e-10 * np.sum(inp.B ** 2)
    assert np.all(np.diff(sigma) <= 1e-12 * sigma[0])          # descending
    assert np.isclose(sigma.sum(), np.sum(inp.B ** 2))          # trace of W


def test_rank_r_integrals_compress_exactly():
    """B^P_ia = sum_r Z_iar C_rP has rank r in the auxiliary index: r NAFs carry it
    all and the pass on them equals the pass on B."""
    rng = np.random.default_rng(3)
    n_h, n_v, n_aux, r = 4, 25, 40, 7
    Z = rng.standard_normal((n_h, n_v, r))
    C = rng.standard_normal((r, n_aux))
    B = 0.05 * np.einsum("iar,rP->iaP", Z, C)
    inp = synth.generate(n_h, 0, n_v, n_aux, seed=3).replace(B=B)
    Bt, sigma, n = naf.naf_compress(B, 1e-10)
    assert n == r
    a = o.pt2_pass_inputs(inp, 0.7)
    b = o.pt2_pass_inputs(inp.replace(B=Bt), 0.7)
    assert abs(a.E - b.E) <= 1e-11 * abs(a.E)
    assert np.abs(a.D_vv - b.D_vv).max() <= 1e-11 * np.abs(a.D_vv).max()


def test_orthogonal_columns_closed_form():
    """J with mutually orthogonal columns: sigma are the squared column norms and
    every NAF is one column (up to sign)."""
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 5)))
    norms = np.array([3.0, 2.0, 1.5, 0.5, 0.1])
    J = Q * norms
    B = J.reshape(3, 20, 5)
    Bt, sigma, n = naf.naf_compress(B, 0.2 / 9.0)
    np.testing.assert_allclose(sigma, norms ** 2, rtol=1e-12)
    assert n == 4
    Jt = Bt.reshape(60, 4)
    for k in range(4):
        assert abs(abs(Jt[:, k] @ J[:, k]) - norms[k] ** 2) <= 1e-12

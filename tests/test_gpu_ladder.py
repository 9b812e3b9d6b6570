"""GPU parity of the particle-particle ladder (pp_ladder) against the FP64 oracle
(oracle/ladder.py), through the C ABI.

Both sides are FP64; the GPU sums in a different order (blocked GEMMs), so the
bar is 1e-12 of the largest |R| (the sums have at most n_aux + n_v^2 terms of
like magnitude: a few hundred ulps).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import ladder
from gpu_common import need_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n_v,n_aux,n_amp", [(70, 90, 5), (33, 17, 3), (1, 5, 2), (96, 40, 2)])
def test_ladder_full_space(n_v, n_aux, n_amp):
    dp = need_gpu()
    inp = synth.ladder_inputs(n_v, n_aux, n_amp, seed=n_v)
    print(f"ladder full n_v={n_v} n_aux={n_aux} n_amp={n_amp}", flush=True)
    ref = ladder.pp_ladder(inp.B_vv, inp.T)
    R = dp.pp_ladder(_dev(inp.B_vv), _dev(inp.T)).cpu().numpy()
    assert np.abs(R - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("n_v,n_kept", [(70, 45), (70, 70), (40, 1)])
def test_ladder_truncated_space(n_v, n_kept):
    dp = need_gpu()
    inp = synth.ladder_inputs(n_v, 50, 4, seed=3)
    q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((n_v, n_v)))
    X = np.ascontiguousarray(q[:, :n_kept])
    print(f"ladder truncated n_v={n_v} n_kept={n_kept}", flush=True)
    ref = ladder.pp_ladder_kept(inp.B_vv, inp.T, X)
    R = dp.pp_ladder(_dev(inp.B_vv), _dev(inp.T), _dev(X), n_kept).cpu().numpy()
    assert R.shape == (4, n_kept, n_kept)
    assert np.abs(R - ref).max() <= TOL * np.abs(ref).max()


def test_ladder_identity_transform_matches_full_space():
    dp = need_gpu()
    inp = synth.ladder_inputs(50, 30, 3, seed=8)
    B, T = _dev(inp.B_vv), _dev(inp.T)
    full = dp.pp_ladder(B, T).cpu().numpy()
    eye = dp.pp_ladder(B, T, _dev(np.eye(50)), 50).cpu().numpy()
    assert np.abs(full - eye).max() <= TOL * np.abs(full).max()


def test_ladder_with_fno_vectors():
    """Kept NOs from the library's own truncation of a density (p_o = 0.985)."""
    dp = need_gpu()
    inp = synth.ladder_inputs(64, 40, 3, seed=2)
    rng = np.random.default_rng(4)
    A = rng.standard_normal((64, 64))
    D = A @ A.T * np.exp(-np.arange(64) / 8.0)[None, :]
    D = 0.5 * (D + D.T)
    t = dp.fno_truncate(_dev(D), 0.985)
    k = t["n_kept"]
    X = t["no_vecs"].cpu().numpy()[:, :k]
    ref = ladder.pp_ladder_kept(inp.B_vv, inp.T, X)
    R = dp.pp_ladder(_dev(inp.B_vv), _dev(inp.T), t["no_vecs"], k).cpu().numpy()  # ldx = n_vir
    assert 1 <= k < 64
    assert np.abs(R - ref).max() <= TOL * np.abs(ref).max()

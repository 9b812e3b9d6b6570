"""CPU pins of the particle-particle ladder oracle (oracle/ladder.py).

The ladder R^p_ab = sum_cd (ac|bd) T^p_cd with (ac|bd) = sum_Q B^Q_ac B^Q_bd is
the N_V^4 contraction of the high-level step (Eq. 6) whose cost the FNO
truncation reduces (Sec. 2).  Pins: explicit loops on tiny sizes, a rank-one
closed form, the per-auxiliary matrix route sum_Q B_Q T B_Q^T (a different order
of the same sums), the transpose symmetry of symmetric DF integrals, covariance
under a full orthogonal change of virtual basis, and the truncated-space ladder
as the projected full-space ladder.
"""
import itertools

import numpy as np

import synth
from oracle import ladder


def _inputs(n_v=9, n_aux=7, n_amp=3, seed=4):
    return synth.ladder_inputs(n_v, n_aux, n_amp, seed)


def test_loops_tiny():
    inp = _inputs(4, 3, 2, seed=1)
    B, T = inp.B_vv, inp.T
    R = ladder.pp_ladder(B, T)
    n = B.shape[0]
    for p, a, b in itertools.product(range(T.shape[0]), range(n), range(n)):
        acc = 0.0
        for c, d, q in itertools.product(range(n), range(n), range(B.shape[2])):
            acc += B[a, c, q] * B[b, d, q] * T[p, c, d]
        assert abs(R[p, a, b] - acc) <= 1e-14 * max(1.0, abs(acc))


def test_rank_one_closed_form():
    rng = np.random.default_rng(3)
    n, n_aux = 8, 5
    u = rng.standard_normal(n)
    B = np.zeros((n, n, n_aux))
    B[:, :, 2] = np.outer(u, u)
    T = rng.standard_normal((2, n, n))
    R = ladder.pp_ladder(B, T)
    for p in range(2):
        np.testing.assert_allclose(R[p], np.outer(u, u) * (u @ T[p] @ u), rtol=1e-13, atol=1e-13)


def test_per_auxiliary_matrix_route():
    inp = _inputs()
    B, T = inp.B_vv, inp.T
    R = ladder.pp_ladder(B, T)
    for p in range(T.shape[0]):
        ref = sum(B[:, :, q] @ T[p] @ B[:, :, q].T for q in range(B.shape[2]))
        np.testing.assert_allclose(R[p], ref, rtol=1e-12, atol=1e-15)


def test_transpose_symmetry():
    inp = _inputs()
    R = ladder.pp_ladder(inp.B_vv, inp.T)
    Rt = ladder.pp_ladder(inp.B_vv, inp.T.transpose(0, 2, 1))
    np.testing.assert_allclose(Rt, R.transpose(0, 2, 1), rtol=1e-12, atol=1e-15)


def test_full_rotation_covariance():
    inp = _inputs()
    q, _ = np.linalg.qr(np.random.default_rng(7).standard_normal((9, 9)))
    R = ladder.pp_ladder(inp.B_vv, inp.T)
    Rk = ladder.pp_ladder_kept(inp.B_vv, inp.T, q)
    np.testing.assert_allclose(Rk, np.einsum("ai,pab,bj->pij", q, R, q), rtol=1e-11, atol=1e-14)


def test_truncated_is_projected_full_ladder():
    inp = _inputs(10, 6, 2, seed=9)
    q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((10, 10)))
    X = q[:, :6]
    P = X @ X.T
    Rk = ladder.pp_ladder_kept(inp.B_vv, inp.T, X)
    Bp = np.einsum("ac,cdQ,db->abQ", P, inp.B_vv, P)
    full = ladder.pp_ladder(Bp, np.einsum("ac,pcd,db->pab", P, inp.T, P))
    np.testing.assert_allclose(Rk, np.einsum("ai,pab,bj->pij", X, full, X), rtol=1e-11, atol=1e-14)
    # the projected integrals vanish outside the kept space
    assert np.abs(ladder.pp_ladder_kept(inp.B_vv, inp.T, q[:, 6:]) -
                  ladder.pp_ladder_kept(Bp, inp.T, q[:, 6:])).max() > 1e-6


def test_generator_symmetry():
    inp = _inputs()
    np.testing.assert_array_equal(inp.B_vv, inp.B_vv.transpose(1, 0, 2))

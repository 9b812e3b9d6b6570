"""CPU pins of the screening oracle: bounds, exact cases, gradients, Adam."""
import math

import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from oracle import screening as sc


def test_bounds_hold_pairwise():
    inp = synth.generate(5, 0, 12, 9, seed=3, localized_xi=2.0)
    s = 0.8
    pq = sc.pair_quantities(inp, s)
    eh, ev = inp.eps_hole, inp.eps_vir
    for p, (i, j) in enumerate(pq["pairs"]):
        V = o.pair_integrals(inp.B, i, j)
        dl = o.pair_denominators(eh, ev, i, j)
        T = o.first_order_doubles(V, dl, s)
        assert np.linalg.norm(V) <= pq["U"][i, j] * (1 + 1e-12)
        g_elem = np.max(np.abs(-np.expm1(-s * dl * dl) / dl))
        g = math.exp(pq["log_gu"][p]) / pq["U"][i, j]
        assert g_elem <= g * (1 + 1e-12)
        assert np.linalg.norm(T) <= math.exp(pq["log_gu"][p]) * (1 + 1e-12)


def test_regularizer_max_against_dense_grid():
    for s, lo, hi in [(0.5, -9.0, -0.5), (1.0, -3.0, -2.5), (2.0, -0.4, -0.1), (0.5, -20.0, -10.0)]:
        d = np.linspace(lo, hi, 400001)
        brute = np.max(-np.expm1(-s * d * d) / np.abs(d))
        assert abs(sc.regularizer_max(s, lo, hi) - brute) <= 1e-8 * brute


def test_w_is_exact_for_orthogonal_rank_one_terms():
    rng = np.random.default_rng(2)
    n_h, n_v, n_aux = 3, 7, 5
    B = np.zeros((n_h, n_v, n_aux))
    rows = rng.permutation(n_v)[:n_aux]
    for Q in range(n_aux):
        B[:, rows[Q], Q] = rng.standard_normal(n_h)
    inp = synth.generate(n_h, 0, n_v, n_aux, seed=1).replace(B=B)
    pq = sc.pair_quantities(inp, 0.5)
    for i in range(n_h):
        for j in range(i, n_h):
            assert abs(np.linalg.norm(o.pair_integrals(B, i, j)) - pq["W"][i, j]) <= 1e-14


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(0)
    w = synth.mlp_init(4) + 0.05 * rng.standard_normal(sc.N_PARAMS)
    X = rng.standard_normal((17, sc.N_IN))
    dout = rng.standard_normal(17)
    out, cache = sc.mlp_forward(w, X)
    g = sc.mlp_backward(w, cache, dout)
    idx = rng.choice(sc.N_PARAMS, 60, replace=False).tolist() + [sc.N_PARAMS - 1, 0, 320, 384, 4480]
    h = 1e-6
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (np.dot(dout, sc.mlp_forward(wp, X)[0]) - np.dot(dout, sc.mlp_forward(wm, X)[0])) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_mse_gradient():
    rng = np.random.default_rng(1)
    out, y = rng.standard_normal(9), rng.standard_normal(9)
    loss, d = sc.mse_and_grad(out, y)
    assert abs(loss - np.mean((out - y) ** 2)) < 1e-15
    h = 1e-7
    for k in range(9):
        op = out.copy()
        op[k] += h
        assert abs((sc.mse_and_grad(op, y)[0] - loss) / h - d[k]) < 1e-6


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    w, m, v = sc.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_fits_a_smooth_target():
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (256, sc.N_IN))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 4]
    w, losses = sc.train(synth.mlp_init(0), X, y, steps=400, lr=3e-3)
    assert losses[-1] < 0.05 * losses[0]


def test_screen_mask():
    pairs = np.array([(0, 0), (0, 1), (1, 1), (0, 2), (1, 2), (2, 2)])
    ln = np.log(np.array([1e-3, 1e-8, 1e-2, 2e-6, 5e-7, 1.0]))
    m = sc.screen_mask(4, pairs, ln, 1e-6)
    assert m[0, 1] == 0 and m[1, 0] == 0 and m[1, 2] == 0 and m[0, 2] == 1
    assert np.array_equal(m, m.T) and m[3].all()
    assert sc.screen_mask(4, pairs, ln, 1e-300).all()

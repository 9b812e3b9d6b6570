"""GPU tests of the learned pair screen: every kernel against the FP64 screening
oracle, training on data the plain pass generates, the rigorous-bound screen,
and what the trained network gains over the method without it."""
import math

import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from oracle import screening as sc
from gpu_common import dd_diff, gpu_pass, need_gpu, torch

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def _features(inp, s):
    dp = need_gpu()
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s)
    f, ls = dp.pairscreen_features(opts, d["eps_hole"], d["eps_vir"], d["B"])
    torch.cuda.synchronize()
    return f, ls


@pytest.mark.parametrize("loc", [None, 1.5])
def test_features_match_oracle(loc):
    inp = synth.generate(9, 0, 70, 130, seed=2, localized_xi=loc)
    f, ls = _features(inp, 0.5)
    ref = sc.pair_quantities(inp, 0.5)
    np.testing.assert_allclose(f.cpu().numpy(), ref["feats"], rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(ls.cpu().numpy()[:, 0], ref["log_gw"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ls.cpu().numpy()[:, 1], ref["log_gu"], rtol=1e-12, atol=1e-12)


def test_forward_backward_adam_match_oracle():
    dp = need_gpu()
    rng = np.random.default_rng(3)
    w = synth.mlp_init(1) + 0.1 * rng.standard_normal(sc.N_PARAMS)
    X = rng.standard_normal((300, 5)).astype(np.float32)
    dout = rng.standard_normal(300).astype(np.float32)
    Wd = _dev(w, torch.float32)
    pred, cache = dp.pairscreen_mlp_forward(Wd, _dev(X, torch.float32), want_cache=True)
    out_ref, cache_ref = sc.mlp_forward(w.astype(np.float32).astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(pred.cpu().numpy(), out_ref, rtol=1e-4, atol=1e-4)
    g = dp.pairscreen_mlp_backward(Wd, _dev(X, torch.float32), cache, _dev(dout, torch.float32))
    g_ref = sc.mlp_backward(w.astype(np.float32).astype(np.float64), cache_ref, dout.astype(np.float64))
    gg = g.cpu().numpy()
    assert np.abs(gg - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
    # one Adam step from zero moments
    m = torch.zeros_like(Wd)
    v = torch.zeros_like(Wd)
    W2 = Wd.clone()
    dp.pairscreen_adam_step(W2, g, m, v, 1, 1e-2)
    w_ref, _, _ = sc.adam_step(w.astype(np.float32).astype(np.float64), gg.astype(np.float64), 0 * w, 0 * w, 1, 1e-2)
    np.testing.assert_allclose(W2.cpu().numpy(), w_ref, rtol=1e-5, atol=1e-6)


def _training_set(n_seeds=60, s=0.5):
    """Plain-pass labels at c1 sizes: half plain inputs, half localized ones."""
    dp = need_gpu()
    feats, ys = [], []
    for k in range(n_seeds):
        xi = None if k % 2 == 0 else float(0.6 + 2.4 * ((k * 37) % 97) / 97.0)
        inp = synth.generate(10, 0, 60, 200, seed=1 + k, localized_xi=xi)
        g = gpu_pass(inp, s)
        d = g["dev"]
        f, ls = dp.pairscreen_features(g["opts"], d["eps_hole"], d["eps_vir"], d["B"])
        y = dp.pairscreen_targets(g["raw"]["pair_tnorm"], ls, inp.n_core, inp.n_h)
        feats.append(f)
        ys.append(y)
    return torch.cat(feats), torch.cat(ys)


def test_targets_and_training():
    dp = need_gpu()
    inp = synth.generate(10, 0, 60, 200, seed=5, localized_xi=1.0)
    g = gpu_pass(inp, 0.5)
    d = g["dev"]
    f, ls = dp.pairscreen_features(g["opts"], d["eps_hole"], d["eps_vir"], d["B"])
    y = dp.pairscreen_targets(g["raw"]["pair_tnorm"], ls, inp.n_core, inp.n_h).cpu().numpy()
    ref = sc.pair_quantities(inp, 0.5)
    r = o.pt2_pass_inputs(inp, 0.5)
    np.testing.assert_allclose(y, sc.targets(r.pair_tnorm, ref["pairs"], ref["log_gw"]), rtol=1e-5, atol=1e-5)
    X, Y = _training_set(40)
    W = _dev(synth.mlp_init(0), torch.float32)
    m, v = torch.zeros_like(W), torch.zeros_like(W)
    losses = dp.pairscreen_train(W, m, v, X, Y, 600, 3e-3).cpu().numpy()
    print("loss first/last", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.1 * losses[0]
    # the same full-batch schedule in FP64 on the CPU reaches a similar loss
    _, lref = sc.train(synth.mlp_init(0), X.cpu().numpy().astype(np.float64), Y.cpu().numpy().astype(np.float64),
                       steps=600, lr=3e-3)
    assert abs(math.log(losses[-1] / lref[-1])) < 0.5


def test_bound_screen_is_rigorous_and_exact_when_empty():
    dp = need_gpu()
    inp = synth.generate(12, 0, 80, 150, seed=9, localized_xi=0.9)
    s, thr = 0.5, 1e-6
    f, ls = _features(inp, s)
    mask, nd = dp.pairscreen_build_mask(None, ls, inp.n_core, inp.n_h, thr, mode=1)
    mk = mask.cpu().numpy()
    r = o.pt2_pass_inputs(inp, s)
    for i in range(inp.n_core):
        for j in range(inp.n_core):
            if mk[i, j] == 0:
                assert r.pair_tnorm[i, j] < thr
    assert nd == (np.sum(mk == 0) + np.sum(np.diag(mk) == 0)) // 2
    # threshold below every bound: nothing dropped, pass identical to the unscreened one
    m0, nd0 = dp.pairscreen_build_mask(None, ls, inp.n_core, inp.n_h, 1e-300, mode=1)
    assert nd0 == 0 and bool((m0 == 1).all())
    a = gpu_pass(inp, s)
    b = gpu_pass(inp, s, pair_mask=m0.cpu().numpy())
    assert a["energy"] == b["energy"] and np.array_equal(a["D"], b["D"])


def test_learned_screen_gain_over_bound():
    """Trained on c1-size plain-pass labels; applied to a larger localized input.
    Both screens must keep the energy within 1e-6 Eh and the kept count of the
    unscreened pass; the network must drop more pairs than the rigorous bound."""
    dp = need_gpu()
    X, Y = _training_set(80)
    W = _dev(synth.mlp_init(0), torch.float32)
    m, v = torch.zeros_like(W), torch.zeros_like(W)
    dp.pairscreen_train(W, m, v, X, Y, 1500, 3e-3)
    resid = (dp.pairscreen_mlp_forward(W, X)[0] - Y).cpu().numpy()
    margin = 4.0 * float(np.std(resid)) + float(np.max(np.abs(resid))) * 0.0
    inp = synth.generate(30, 0, 150, 500, seed=21, localized_xi=1.25)
    s, thr, p_o = 0.5, 1e-6, 0.985
    f, ls = _features(inp, s)
    pred, _ = dp.pairscreen_mlp_forward(W, f)
    m_net, nd_net = dp.pairscreen_build_mask(pred, ls, inp.n_core, inp.n_h, thr, margin, 0)
    m_bnd, nd_bnd = dp.pairscreen_build_mask(None, ls, inp.n_core, inp.n_h, thr, 0.0, 1)
    full = gpu_pass(inp, s)
    net = gpu_pass(inp, s, pair_mask=m_net.cpu().numpy())
    bnd = gpu_pass(inp, s, pair_mask=m_bnd.cpu().numpy())
    print(f"pairs {inp.n_core * (inp.n_core + 1) // 2}: dropped by network {nd_net}, by bound {nd_bnd}; "
          f"dE net {dd_diff(net['energy'], full['energy']):.2e} bound {dd_diff(bnd['energy'], full['energy']):.2e}",
          flush=True)
    r = o.pt2_pass_inputs(inp, s)
    truth_below = np.sum(np.triu(r.pair_tnorm[:30, :30] < thr))
    assert nd_net >= nd_bnd and nd_net > 0 and nd_net <= truth_below
    # pair by pair: every pair either screen drops is truly below the threshold
    for mk in (m_net.cpu().numpy(), m_bnd.cpu().numpy()):
        wrong = [(i, j, r.pair_tnorm[i, j]) for i in range(inp.n_core) for j in range(i, inp.n_core)
                 if mk[i, j] == 0 and not r.pair_tnorm[i, j] < thr]
        assert not wrong, wrong[:5]
    for g in (net, bnd):
        assert dd_diff(g["energy"], full["energy"]) <= 1e-6
        t0 = dp.fno_truncate(full["raw"]["D_vv"], p_o)
        t1 = dp.fno_truncate(g["raw"]["D_vv"], p_o)
        assert t0["n_kept"] == t1["n_kept"]
        assert np.abs(t0["occ"].cpu().numpy() - t1["occ"].cpu().numpy()).max() <= 1e-9 * t0["occ"].max().item()

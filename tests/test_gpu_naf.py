"""GPU parity of the natural-auxiliary-function compression (naf_compress) against
the oracle (oracle/naf.py), and the pass run on the compressed integrals."""
import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from oracle import naf
from gpu_common import dd_diff, gpu_pass, need_gpu, torch

pytestmark = pytest.mark.gpu

E_TOL = 1e-8


def _run(inp, eps):
    dp = need_gpu()
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, 0.5)
    r = dp.naf_compress(opts, d["B"], eps)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("sizes,loc", [((10, 0, 60, 200), None), ((6, 4, 50, 90), 1.5), ((3, 0, 70, 130), None)])
def test_naf_eigenvalues_count_and_pass(sizes, loc):
    inp = synth.generate(*sizes, seed=7, localized_xi=loc)
    print(f"sizes={sizes} loc={loc}", flush=True)
    Bt_ref, sig_ref, _ = naf.naf_compress(inp.B, 0.0)
    r = _run(inp, 0.0)
    assert r["n_naf"] == inp.n_aux
    sig = r["sigma"].cpu().numpy()
    assert np.abs(sig - sig_ref).max() <= 1e-11 * sig_ref[0]
    # every function kept: the pass on B~ is the pass on B
    full = o.pt2_pass_inputs(inp, 0.5)
    g = gpu_pass(inp.replace(B=r["B_naf"].cpu().numpy()), 0.5)
    assert dd_diff(g["energy"], full.energy) <= E_TOL
    assert np.abs(g["D"] - full.D_vv).max() <= 1e-11 * np.abs(full.D_vv).max()
    # truncating thresholds between eigenvalues: the same count and the same compressed pass
    for k in (inp.n_aux // 2, inp.n_aux // 5):
        eps = 0.5 * (sig_ref[k - 1] + sig_ref[k]) / sig_ref[0]
        r = _run(inp, eps)
        Bt, _, nk = naf.naf_compress(inp.B, eps)
        assert r["n_naf"] == nk == k
        ref = o.pt2_pass_inputs(inp.replace(B=Bt), 0.5)
        g = gpu_pass(inp.replace(B=r["B_naf"].cpu().numpy()), 0.5)
        print(f"  n_naf {k}: E {ref.E:.8f} (full {full.E:.8f}), GPU dE {dd_diff(g['energy'], ref.energy):.2e}",
              flush=True)
        assert dd_diff(g["energy"], ref.energy) <= E_TOL
        assert np.abs(g["D"] - ref.D_vv).max() <= 1e-10 * np.abs(ref.D_vv).max()


def test_naf_threshold_above_all_rejected():
    dp = need_gpu()
    inp = synth.generate(2, 0, 20, 30, seed=1)
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, 0.5)
    with pytest.raises(dp.DfptError):
        dp.naf_compress(opts, d["B"], 2.0)


def test_naf_redundant_auxiliary_set():
    """A rank-r auxiliary set up to 1e-7 noise: the relative threshold 1e-8 keeps r
    functions, eigenvectors are formed only for them (the near-zero cluster is
    skipped), and the pass on the compressed integrals matches the oracle's."""
    inp = synth.generate(6, 0, 80, 300, seed=2, aux_rank=40, aux_noise=1e-7)
    r = _run(inp, 1e-8)
    Bt, sig, nk = naf.naf_compress(inp.B, 1e-8)
    assert r["n_naf"] == nk == 40
    full = o.pt2_pass_inputs(inp, 0.5)
    g = gpu_pass(inp.replace(B=r["B_naf"].cpu().numpy()), 0.5)
    print(f"  redundant set: dE vs uncompressed {dd_diff(g['energy'], full.energy):.2e}", flush=True)
    assert dd_diff(g["energy"], o.pt2_pass_inputs(inp.replace(B=Bt), 0.5).energy) <= E_TOL
    assert dd_diff(g["energy"], full.energy) <= 1e-6 * abs(full.E)

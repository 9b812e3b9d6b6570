"""dfpt2_build_vv_density_noalloc (the pass in the library's static scratch, for
callers that cannot allocate) against dfpt2_build_vv_density with a caller
workspace: two calls in a row, the second on smaller inputs, in FP64 and in split
BF16, each compared with the workspace entry point on the same inputs at the
bar of the parity tests (same energy to 1e-12 relative, same D_vv, same pair
data); and a pass larger than the scratch returns DFPT2_ERR_WORKSPACE."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import dd_diff, need_gpu

pytestmark = pytest.mark.gpu


def _both(dp, inp, precision, s=0.5):
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s, precision=precision)
    ref = dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], want_pair_energy=True,
                              want_pair_tnorm=True)
    n_h, n_v = inp.n_h, inp.n_vir
    out = dict(D_vv=torch.full((n_v, n_v), float("nan"), dtype=torch.float64, device="cuda"),
               e_pt2=torch.full((2,), float("nan"), dtype=torch.float64, device="cuda"),
               pair_energy=torch.full((n_h, n_h), float("nan"), dtype=torch.float64, device="cuda"),
               pair_tnorm=torch.full((n_h, n_h), float("nan"), dtype=torch.float32, device="cuda"))
    r = dp.build_vv_density_noalloc(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], **out)
    torch.cuda.synchronize()
    return ref, r


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "bf16"])
def test_noalloc_matches_workspace_entry_point(precision):
    dp = need_gpu()
    for k, sizes in enumerate(((10, 0, 60, 200), (6, 2, 37, 50))):
        inp = synth.generate(*sizes, seed=5 + k)
        print(f"noalloc: call {k + 1}, sizes {sizes}, precision {precision}", flush=True)
        ref, r = _both(dp, inp, precision)
        e0 = tuple(float(x) for x in ref["e_pt2"].cpu().numpy())
        e1 = tuple(float(x) for x in r["e_pt2"].cpu().numpy())
        assert dd_diff(e0, e1) <= 1e-12 * abs(e0[0])
        D0, D1 = ref["D_vv"].cpu().numpy(), r["D_vv"].cpu().numpy()
        assert np.abs(D0 - D1).max() <= 1e-12 * np.abs(D0).max()
        pe0, pe1 = ref["pair_energy"].cpu().numpy(), r["pair_energy"].cpu().numpy()
        fin = np.isfinite(pe0)
        assert np.array_equal(fin, np.isfinite(pe1))
        assert np.abs(pe0[fin] - pe1[fin]).max() <= 1e-12 * np.abs(pe0[fin]).max()
        np.testing.assert_allclose(r["pair_tnorm"].cpu().numpy(), ref["pair_tnorm"].cpu().numpy(), rtol=1e-6)


def test_noalloc_rejects_a_pass_beyond_the_scratch():
    dp = need_gpu()
    from paper_2312_07008_amd._lib import ERR_WORKSPACE, STATIC_SCRATCH_BYTES, DfptError
    inp = synth.generate(20, 0, 128, 300, seed=1)
    opts = dp.make_opts(20, 0, 128, 300, 0.5, precision=dp.BF16_SLICED)
    assert dp.workspace_size(opts) > STATIC_SCRATCH_BYTES
    d = dp.upload_inputs(inp)
    D = torch.zeros((128, 128), dtype=torch.float64, device="cuda")
    e = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(DfptError) as ex:
        dp.build_vv_density_noalloc(opts, d["eps_hole"], d["eps_vir"], None, d["B"], D_vv=D, e_pt2=e)
    assert ex.value.status == ERR_WORKSPACE
    assert float(D.abs().max()) == 0.0 and float(e.abs().max()) == 0.0
    # a smaller pair batch brings the same pass under the limit, with the same energy
    opts_b = dp.make_opts(20, 0, 128, 300, 0.5, precision=dp.BF16_SLICED, pair_batch=16)
    assert dp.workspace_size(opts_b) <= STATIC_SCRATCH_BYTES
    dp.build_vv_density_noalloc(opts_b, d["eps_hole"], d["eps_vir"], None, d["B"], D_vv=D, e_pt2=e)
    ref = dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], None, d["B"])
    torch.cuda.synchronize()
    e0 = tuple(float(x) for x in ref["e_pt2"].cpu().numpy())
    e1 = tuple(float(x) for x in e.cpu().numpy())
    assert dd_diff(e0, e1) <= 1e-12 * abs(e0[0])

"""Helpers shared by the GPU tests: run the HIP path through the C ABI and bring
results back as numpy arrays.  The oracle is never called from here."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_07008_amd as dp
    dp.load()
    return dp


def gpu_pass(inp, s, precision=0, pair_mask=None, **kw):
    dp = need_gpu()
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s, precision=precision, **kw)
    mask = None
    if pair_mask is not None:
        mask = torch.from_numpy(np.ascontiguousarray(pair_mask.astype(np.uint8))).cuda()
    r = dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], mask,
                            want_pair_energy=True, want_pair_tnorm=True)
    torch.cuda.synchronize()
    e = r["e_pt2"].cpu().numpy()
    return dict(energy=(float(e[0]), float(e[1])), E=float(e[0]) + float(e[1]),
                D=r["D_vv"].cpu().numpy(), pair_energy=r["pair_energy"].cpu().numpy(),
                pair_tnorm=r["pair_tnorm"].cpu().numpy(), dev=d, opts=opts, raw=r)


def dd_diff(a, b):
    """|a - b| for two double-doubles, evaluated without cancellation loss."""
    import math
    return abs(math.fsum([a[0], a[1], -b[0], -b[1]]))

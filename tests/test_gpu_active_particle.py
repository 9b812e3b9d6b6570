"""GPU parity of the Eq. A9 terms with an active particle index
(dfpt2_add_active_particle_density) against the FP64 oracle (oracle/a9_active.py),
through the C ABI.  FP64 on both sides; bar 1e-11 of max|D| (GEMM sums in a
different order over n_aux and n_h^2 n_act terms)."""
import numpy as np
import pytest
import torch

import synth
from oracle import a9_active
from oracle import dsrg_pt2 as o
from gpu_common import need_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _run(inp, s, density_convention=0, base=None):
    dp = need_gpu()
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s, density_convention=density_convention)
    D = torch.zeros((inp.n_vir, inp.n_vir), dtype=torch.float64, device="cuda") if base is None else base
    dp.add_active_particle_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], d["B_act"], D)
    torch.cuda.synchronize()
    return D.cpu().numpy(), d, opts


@pytest.mark.parametrize("sizes,s", [((6, 4, 90, 140), 0.5), ((1, 2, 33, 17), 1.0), ((0, 6, 70, 50), 0.7),
                                     ((12, 8, 130, 96), 0.5)])
def test_active_particle_terms_parity(sizes, s):
    inp = synth.generate(*sizes, seed=3, active_particles=True)
    print(f"active-particle terms sizes={sizes} s={s}", flush=True)
    ref = a9_active.active_particle_density(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B,
                                            inp.B_act, s)
    D, _, _ = _run(inp, s)
    assert np.abs(D - ref).max() <= TOL * np.abs(ref).max()
    assert np.array_equal(D, D.T)


def test_added_to_the_pass_density_and_per_spin():
    dp = need_gpu()
    inp = synth.generate(5, 4, 80, 100, seed=4, active_particles=True)
    s = 0.5
    ref = (o.pt2_pass_inputs(inp, s).D_vv +
           a9_active.active_particle_density(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B,
                                             inp.B_act, s))
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s)
    r = dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"])
    D = dp.add_active_particle_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], d["B_act"],
                                       r["D_vv"]).cpu().numpy()
    assert np.abs(D - ref).max() <= TOL * np.abs(ref).max()
    half, _, _ = _run(inp, s, density_convention=1)
    full, _, _ = _run(inp, s)
    np.testing.assert_allclose(half, 0.5 * full, rtol=1e-15, atol=0)


def test_closed_shell_adds_nothing():
    inp = synth.generate(4, 0, 40, 30, seed=5)
    dp = need_gpu()
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(4, 0, 40, 30, 0.5)
    D = torch.ones((40, 40), dtype=torch.float64, device="cuda")
    dp.add_active_particle_density(opts, d["eps_hole"], d["eps_vir"], d["eps_vir"][:0], d["B"], d["B"][:0], D)
    assert float(D.sum()) == 1600.0

"""GPU parity of dfpt2_add_cumulant_singles_density (the singles of Eq. A6 and the
Eq. A9 terms with the singles and the two-body cumulant) against the FP64 oracle
(oracle/a9_cumulant.py), through the C ABI: several sizes that span MFMA tiles,
ragged edges and the no-core and one-core cases, with and without the cumulant,
per-spin convention, and the singles amplitudes themselves.  End to end, on a
correlated reference (a two-state singlet ensemble of the active orbitals), the
three D_vv entry points of the library plus the dropped three-body-cumulant term
equal the exact 1/2 Tr(rho [[E_ef, A], A]) of a Fock-space evaluation."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import need_gpu
from oracle import a9_cumulant as cu

pytestmark = pytest.mark.gpu

CASES = [((2, 2, 30, 40), 1, 0.7), ((3, 4, 70, 90), 2, 0.5), ((5, 4, 129, 77), 3, 1.1), ((0, 4, 50, 60), 4, 0.5),
         ((1, 2, 33, 17), 5, 0.9), ((20, 6, 131, 140), 6, 0.5)]


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float64)


def _run(dp, inp, lam, s, convention=0):
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s, density_convention=convention)
    D = torch.zeros((inp.n_vir, inp.n_vir), dtype=torch.float64, device="cuda")
    t1 = torch.zeros((inp.n_h, inp.n_vir), dtype=torch.float64, device="cuda")
    dp.add_cumulant_singles_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"],
                                    None if lam is None else _dev(lam), d["B"], d["B_act"], D, t1=t1)
    torch.cuda.synchronize()
    return D.cpu().numpy(), t1.cpu().numpy()


@pytest.mark.parametrize("sizes,seed,s", CASES, ids=[f"{c[0]}" for c in CASES])
def test_cumulant_singles_parity(sizes, seed, s):
    dp = need_gpu()
    print(f"cumulant/singles: sizes {sizes} seed {seed} s {s}", flush=True)
    inp = synth.generate(*sizes, seed=seed, active_particles=True)
    lam = synth.active_cumulant(inp.n_act, seed)
    D, t1 = _run(dp, inp, lam, s)
    ref = cu.cumulant_singles_density(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, lam, inp.B, inp.B_act, s)
    t1_ref = cu.singles_amplitudes(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B, inp.B_act, s)
    scale = np.abs(ref).max()
    print(f"  max|D| {scale:.3e}, max|dD| {np.abs(D - ref).max():.3e}, max|dt1| {np.abs(t1 - t1_ref).max():.3e}",
          flush=True)
    assert np.abs(D - ref).max() <= 1e-12 * scale
    assert np.array_equal(D, D.T)
    assert np.abs(t1 - t1_ref).max() <= 1e-13 * np.abs(t1_ref).max()
    # without a cumulant: the singles terms alone; per-spin convention: half
    D1, _ = _run(dp, inp, None, s)
    ref1 = cu.cumulant_singles_density(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, lam, inp.B, inp.B_act, s,
                                       terms=[1])
    assert np.abs(D1 - ref1).max() <= 1e-12 * np.abs(ref1).max()
    Dh, _ = _run(dp, inp, lam, s, convention=1)
    assert np.abs(Dh - 0.5 * ref).max() <= 1e-12 * scale


def test_no_active_orbitals_adds_nothing():
    dp = need_gpu()
    inp = synth.generate(4, 0, 40, 30, seed=7)
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(4, 0, 40, 30, 0.5)
    D = torch.full((40, 40), 3.0, dtype=torch.float64, device="cuda")
    Bact = torch.zeros(0, dtype=torch.float64, device="cuda")
    g = torch.zeros(0, dtype=torch.float64, device="cuda")
    dp.add_cumulant_singles_density(opts, d["eps_hole"], d["eps_vir"], g, None, d["B"], Bact, D)
    torch.cuda.synchronize()
    assert bool((D == 3.0).all())


@pytest.mark.parametrize("sizes,seed", [((1, 2, 2, 3), 1), ((2, 2, 3, 4), 8)])
def test_all_of_eq_a9_against_fock_space(sizes, seed):
    """build_vv_density + add_active_particle_density + add_cumulant_singles_density on
    a correlated reference, plus the three-body-cumulant term (not part of the method,
    from the oracle), equal the exact second-order virtual 1-RDM."""
    dp = need_gpu()
    from fock_bruteforce import active_rdms, brute_force_pt2, singlet_pair_states
    inp = synth.generate(*sizes, seed=seed, active_particles=True)
    inp = inp.replace(B=inp.B * 7.0, B_act=inp.B_act * 7.0)
    s = 0.7
    rng = np.random.default_rng(seed + 100)
    states = singlet_pair_states(inp.n_act, [rng.standard_normal((inp.n_act, inp.n_act)) for _ in range(2)])
    w = list(rng.dirichlet(np.ones(2)))
    g, l2, l3, _ = active_rdms(inp.n_act, w, states)
    inp = inp.replace(gamma_act=g)
    t1 = cu.singles_amplitudes(inp.eps_core, inp.eps_act, inp.eps_vir, g, inp.B, inp.B_act, s)
    _, G, _ = brute_force_pt2(inp.eps_core, inp.eps_act, inp.eps_vir, g, inp.B, s, B_act=inp.B_act,
                              states=(w, states), singles=t1)
    d = dp.upload_inputs(inp)
    opts = dp.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s)
    r = dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"])
    D = r["D_vv"]
    dp.add_active_particle_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], d["B_act"], D)
    dp.add_cumulant_singles_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], _dev(l2), d["B"], d["B_act"], D)
    torch.cuda.synchronize()
    tot = D.cpu().numpy() + cu.three_cumulant_term(inp.eps_core, inp.eps_act, inp.eps_vir, inp.B, inp.B_act, l3, s)
    print(f"  max|G| {np.abs(G).max():.3e}, max|GPU - G| {np.abs(tot - G).max():.3e}", flush=True)
    assert np.abs(tot - G).max() <= 1e-12 * np.abs(G).max()

"""CPU pins of the singles (Eq. A6) and the density-cumulant terms of Eq. A9
(oracle/a9_cumulant.py), evaluated from first principles in a tiny Fock space.

* The bracket of Eq. A6 (f = 0) is the one-body part of [H0, T2], the first-order
  source of the singles: read off a quasi-free reference with a non-diagonal
  active density by the generalized Wick theorem (tests/fock_bruteforce.py).
* On correlated references -- ensembles of two-electron singlet states of the
  active orbitals, whose 2- and 3-cumulants are far from zero -- the exact
  1/2 Tr(rho [[E_ef, A], A]) with singles and doubles in A equals the terms of
  oracle.dsrg_pt2, oracle.a9_active and oracle.a9_cumulant plus the three-body
  cumulant term the method drops (Sec. 2), evaluated from the same ensemble.
  An alternative reading of the P shorthand, or any term left out, fails it.
* Closed forms: a density diagonal in the semicanonical basis gives no singles
  (Delta_u^u = 0); a single determinant has no cumulants.
"""
import numpy as np
import pytest

import synth
from fock_bruteforce import active_rdms, brute_force_pt2, singlet_pair_states
from oracle import a9_active, a9_cumulant as cu
from oracle import dsrg_pt2 as o


def _inputs(sizes, seed):
    inp = synth.generate(*sizes, seed=seed, active_particles=True)
    return inp.replace(B=inp.B * 7.0, B_act=inp.B_act * 7.0)   # O(1) amplitudes


def _ensemble(n_act, seed, n_states=2):
    rng = np.random.default_rng(seed + 100)
    states = singlet_pair_states(n_act, [rng.standard_normal((n_act, n_act)) for _ in range(n_states)])
    w = list(rng.dirichlet(np.ones(n_states)))
    return w, states


@pytest.mark.parametrize("sizes,seed", [((1, 2, 2, 3), 1), ((0, 2, 2, 3), 3), ((1, 2, 1, 2), 4),
                                        ((2, 2, 1, 3), 2)])
def test_singles_source_is_the_one_body_part_of_H0_T2(sizes, seed):
    inp = _inputs(sizes, seed)
    s = 0.7
    src = brute_force_pt2(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B, s, B_act=inp.B_act,
                          probe_singles_source=True)
    ref = cu.singles_source(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B, inp.B_act, s)
    assert np.abs(ref).max() > 1e-5
    for sig in range(2):
        np.testing.assert_allclose(src[..., sig], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _full_density(inp, g, l2, l3, s, terms=None):
    inp = inp.replace(gamma_act=g)
    D0 = o.pt2_pass_inputs(inp, s).D_vv
    D1 = a9_active.active_particle_density(inp.eps_core, inp.eps_act, inp.eps_vir, g, inp.B, inp.B_act, s)
    D2 = cu.cumulant_singles_density(inp.eps_core, inp.eps_act, inp.eps_vir, g, l2, inp.B, inp.B_act, s,
                                     terms=terms)
    D3 = cu.three_cumulant_term(inp.eps_core, inp.eps_act, inp.eps_vir, inp.B, inp.B_act, l3, s)
    return D0 + D1 + D2 + D3


def _brute(inp, w, states, g, s):
    t1 = cu.singles_amplitudes(inp.eps_core, inp.eps_act, inp.eps_vir, g, inp.B, inp.B_act, s)
    _, G, gam = brute_force_pt2(inp.eps_core, inp.eps_act, inp.eps_vir, g, inp.B, s, B_act=inp.B_act,
                                states=(w, states), singles=t1)
    np.testing.assert_allclose(gam, g, atol=1e-13)
    return G


@pytest.mark.parametrize("sizes,seed,s", [((1, 2, 2, 3), 1, 0.7), ((0, 2, 2, 3), 3, 0.7), ((1, 2, 1, 2), 4, 1.3),
                                          ((2, 2, 1, 3), 2, 0.4), ((2, 2, 2, 2), 5, 0.7)])
def test_correlated_reference_brute_force(sizes, seed, s):
    inp = _inputs(sizes, seed)
    w, states = _ensemble(inp.n_act, seed)
    g, l2, l3, _ = active_rdms(inp.n_act, w, states)
    assert np.abs(l2).max() > 0.1 and np.abs(l3).max() > 0.01          # a correlated reference
    G = _brute(inp, w, states, g, s)
    D = _full_density(inp, g, l2, l3, s)
    np.testing.assert_allclose(D, G, rtol=0, atol=1e-12 * np.abs(G).max())
    # every term matters at this size, and leaving one out breaks the match
    for k in range(1, 7):
        Dk = _full_density(inp, g, l2, l3, s, terms=[j for j in range(1, 7) if j != k])
        if np.abs(D - Dk).max() > 1e-10 * np.abs(G).max():
            assert np.abs(Dk - G).max() > 1e-10 * np.abs(G).max()


def test_alternative_readings_of_P_fail():
    """The fourth product of P trades the second particle index of the first amplitude
    with the second hole index of the second and swaps the hole pairs of both
    (- t_{aq}^{ji} t_{cd}^{pk}).  Without it, or with it but the first amplitude's holes
    left unswapped (- t_{aq}^{ij} t_{cd}^{pk}), the correlated brute force is missed."""
    inp = _inputs((1, 2, 2, 3), 1)
    s = 0.7
    w, states = _ensemble(inp.n_act, 1)
    g, l2, l3, _ = active_rdms(inp.n_act, w, states)
    G = _brute(inp, w, states, g, s)
    good = _full_density(inp, g, l2, l3, s)
    assert np.abs(good - G).max() <= 1e-12 * np.abs(G).max()
    n_core = inp.n_core
    eps_h = np.concatenate([inp.eps_core, inp.eps_act])
    X, _ = cu._amplitude_blocks(eps_h, inp.eps_act, inp.eps_vir, inp.B, inp.B_act, s)
    Xca, Xac, Xaa = X[:n_core, n_core:], X[n_core:, :n_core], X[n_core:, n_core:]
    # the fourth products as the oracle forms them (D4: sum over core m; D6: with gamma)
    fourth = sum(np.einsum("vex,yfu,uvxy->ef", Xac[:, m], Xac[:, m], l2) for m in range(n_core))
    fourth = fourth + 0.5 * np.einsum("vwex,yzfu,wz,uvxy->ef", Xaa, Xaa, g, l2)
    unswapped = sum(np.einsum("vex,yfu,uvxy->ef", Xca[m], Xac[:, m], l2) for m in range(n_core))
    unswapped = unswapped + 0.5 * np.einsum("wvex,yzfu,wz,uvxy->ef", Xaa, Xaa, g, l2)
    v1 = good + fourth                      # fourth product left out (it enters with a minus sign)
    v2 = good + fourth - unswapped          # first amplitude's holes not swapped
    for v in (v1, v2):
        assert np.abs(v - G).max() > 1e-6 * np.abs(G).max()


def test_diagonal_density_gives_no_singles():
    """Gamma diagonal in the semicanonical basis: gamma_x^u Delta_u^x = n_u delta_ux
    (eps_u - eps_u) = 0, so Eq. A6 has no source without f."""
    inp = _inputs((2, 2, 4, 5), 9)
    src = cu.singles_source(inp.eps_core, inp.eps_act, inp.eps_vir, np.diag([1.6, 0.3]), inp.B, inp.B_act, 0.5)
    assert np.abs(src).max() == 0.0


def test_determinant_has_no_cumulants_and_reduces_to_zero_cumulant_terms():
    """One closed-shell determinant in the active space: lambda_2 = lambda_3 = 0, and the
    brute force equals the zero-cumulant terms plus the singles."""
    inp = _inputs((1, 2, 2, 3), 6)
    s = 0.7
    states = singlet_pair_states(2, [np.array([[1.0, 0.0], [0.0, 0.0]])])
    g, l2, l3, _ = active_rdms(2, [1.0], states)
    assert np.abs(l2).max() < 1e-14 and np.abs(l3).max() < 1e-14
    G = _brute(inp, [1.0], states, g, s)
    D = _full_density(inp, g, l2, l3, s)
    np.testing.assert_allclose(D, G, rtol=0, atol=1e-12 * np.abs(G).max())


def test_terms_are_symmetric():
    inp = _inputs((1, 2, 3, 4), 7)
    w, states = _ensemble(2, 7)
    g, l2, _, _ = active_rdms(2, w, states)
    for k in range(1, 7):
        Dk = cu.cumulant_singles_density(inp.eps_core, inp.eps_act, inp.eps_vir, g, l2, inp.B, inp.B_act, 0.5,
                                         terms=[k])
        assert np.abs(Dk - Dk.T).max() <= 1e-14 * max(np.abs(Dk).max(), 1e-300)

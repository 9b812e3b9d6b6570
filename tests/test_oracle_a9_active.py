"""CPU pins of the Eq. A9 terms with an active particle index (oracle/a9_active.py).

The pin is an evaluation from first principles: in a tiny Fock space, with the
particle indices of the (normal-ordered) doubles running over active and virtual
orbitals, 1/2 Tr(rho [[E_ef, A], A]) over a quasi-free reference equals the
three terms with two virtual particle indices (oracle.dsrg_pt2) plus the three
zero-cumulant terms with one active particle index (oracle.a9_active), for
diagonal and non-diagonal active densities.  Limits: an empty active space
(Gamma = 0) turns the active orbitals into virtuals, and a full one (Gamma = 2)
into core orbitals, where the active-particle terms vanish (eta = 0).
"""
import numpy as np
import pytest

import synth
from fock_bruteforce import brute_force_pt2
from oracle import a9_active
from oracle import dsrg_pt2 as o


def _inputs(sizes, seed, gamma=None):
    inp = synth.generate(*sizes, seed=seed, active_particles=True)
    inp = inp.replace(B=inp.B * 7.0, B_act=inp.B_act * 7.0)   # O(1) amplitudes
    if gamma is not None:
        inp = inp.replace(gamma_act=gamma)
    return inp


def _total(inp, s):
    r = o.pt2_pass_inputs(inp, s)
    extra = a9_active.active_particle_density(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B,
                                              inp.B_act, s)
    return r.D_vv, extra


@pytest.mark.parametrize("sizes,seed", [((1, 2, 2, 3), 1), ((2, 2, 1, 3), 2), ((0, 2, 2, 3), 3),
                                        ((1, 2, 1, 2), 4)])
def test_fock_space_brute_force_with_active_particles(sizes, seed):
    inp = _inputs(sizes, seed)
    s = 0.7
    _, G, gam = brute_force_pt2(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B, s, B_act=inp.B_act)
    np.testing.assert_allclose(gam, inp.gamma_act, atol=1e-13)
    D_vv, extra = _total(inp, s)
    assert np.abs(extra).max() > 1e-3 * np.abs(G).max()          # the terms matter here
    np.testing.assert_allclose(D_vv + extra, G, rtol=0, atol=1e-12 * np.abs(G).max())


def test_brute_force_diagonal_fractional_density():
    inp = _inputs((1, 2, 2, 3), 5, gamma=np.diag([0.4, 1.3]))
    s = 1.1
    _, G, _ = brute_force_pt2(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B, s, B_act=inp.B_act)
    D_vv, extra = _total(inp, s)
    np.testing.assert_allclose(D_vv + extra, G, rtol=0, atol=1e-12 * np.abs(G).max())


def test_empty_active_space_is_virtual():
    """Gamma = 0: the active orbitals are empty; the active-particle terms are then the
    core-core term with those orbitals as extra virtual particles, 2 t tc^T summed over x."""
    inp = _inputs((3, 2, 5, 4), 6, gamma=np.zeros((2, 2)))
    s = 0.5
    extra = a9_active.active_particle_density(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B,
                                              inp.B_act, s)
    eps_h = np.concatenate([inp.eps_core, inp.eps_act])
    want = np.zeros((5, 5))
    for m in range(3):
        for n in range(3):
            Xmn = a9_active.active_particle_amplitudes(eps_h, inp.eps_act, inp.eps_vir, inp.B, inp.B_act, m, n, s)
            Xnm = a9_active.active_particle_amplitudes(eps_h, inp.eps_act, inp.eps_vir, inp.B, inp.B_act, n, m, s)
            want += 2.0 * Xmn @ (2.0 * Xmn - Xnm).T
    np.testing.assert_allclose(extra, want, rtol=1e-13, atol=1e-16)


def test_full_active_space_terms_vanish():
    inp = _inputs((2, 2, 4, 3), 7, gamma=2.0 * np.eye(2))
    extra = a9_active.active_particle_density(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B,
                                              inp.B_act, 0.5)
    assert np.abs(extra).max() == 0.0


def test_active_rotation_invariance():
    """Rotating the active orbitals (Gamma, B_act's hole and particle indices, with equal
    active energies so the rotation keeps them semicanonical) leaves the terms unchanged."""
    base = synth.generate(2, 2, 4, 5, seed=8, active_particles=True)
    eps_act = np.full(2, -0.15)
    q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((2, 2)))
    Ba = base.B_act.copy()
    Ba2 = np.einsum("xy,iyQ->ixQ", q.T, Ba)                      # particle index
    Ba2[2:] = np.einsum("uv,vxQ->uxQ", q.T, Ba2[2:])              # active hole index
    B2 = base.B.copy()
    B2[2:] = np.einsum("uv,vaQ->uaQ", q.T, B2[2:])
    G2 = q.T @ base.gamma_act @ q
    d1 = a9_active.active_particle_density(base.eps_core, eps_act, base.eps_vir, base.gamma_act, base.B, Ba, 0.5)
    d2 = a9_active.active_particle_density(base.eps_core, eps_act, base.eps_vir, G2, B2, Ba2, 0.5)
    np.testing.assert_allclose(d2, d1, rtol=1e-12, atol=1e-16)

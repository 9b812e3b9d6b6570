"""CPU pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a second-
quantized brute force, a textbook limit, a finite-difference derivative, an
invariance, a closed form or a hand-made spectrum.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dsrg_pt2 as o
from fock_bruteforce import brute_force_pt2


def _closed(n_occ, n_vir, n_aux, seed=0):
    return synth.generate(n_occ, 0, n_vir, n_aux, seed)


# ---------------------------------------------------------------------------
# Second-quantized brute force (App. A, Eqs. A4, A7, A8, A9)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sizes,seed,s", [((2, 0, 3, 4), 3, 0.7), ((1, 0, 3, 5), 1, 2.0),
                                          ((1, 2, 2, 3), 3, 0.7), ((0, 2, 3, 3), 5, 0.4),
                                          ((1, 2, 3, 3), 7, 1.3)])
def test_fock_space_brute_force(sizes, seed, s):
    inp = synth.generate(*sizes, seed=seed)
    inp = inp.replace(B=inp.B * 7.0)           # O(1) amplitudes for a relative check
    E2, G, gam = brute_force_pt2(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B, s)
    if inp.n_act:
        np.testing.assert_allclose(gam, inp.gamma_act, atol=1e-13)
    r = o.pt2_pass_inputs(inp, s)
    assert abs(r.E - E2) <= 1e-12 * abs(E2)
    np.testing.assert_allclose(r.D_vv, G, rtol=0, atol=1e-12 * np.abs(G).max())


# ---------------------------------------------------------------------------
# Single-reference limit s -> infinity is MP2 (App. A, last paragraph)
# ---------------------------------------------------------------------------

def _textbook_mp2_closed_shell(inp):
    """E_MP2 = sum_{ijab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b)."""
    ia_jb = np.einsum("iaQ,jbQ->iajb", inp.B, inp.B)
    e_o, e_v = inp.eps_core, inp.eps_vir
    den = e_o[:, None, None, None] + e_o[None, None, :, None] - e_v[None, :, None, None] - e_v[None, None, None, :]
    ib_ja = ia_jb.transpose(0, 3, 2, 1)
    return float(np.sum(ia_jb * (2.0 * ia_jb - ib_ja) / den))


def test_mp2_limit_energy():
    inp = synth.config_inputs("c1")
    r = o.pt2_pass_inputs(inp, 1e3, with_density=False)   # e^{-s D^2} underflows to 0
    e_mp2 = _textbook_mp2_closed_shell(inp)
    assert abs(r.E - e_mp2) <= 1e-12 * abs(e_mp2)


def test_mp2_limit_density_is_energy_derivative_diagonal():
    """Gamma = dE/df (Eq. 7): in the MP2 limit the amplitudes are stationary, so the
    diagonal of D equals the total derivative of E with respect to eps_e."""
    inp = _closed(3, 7, 11, seed=4)
    s = 1e3
    r = o.pt2_pass_inputs(inp, s)
    h = 1e-5
    for e in range(inp.n_vir):
        ep, em = inp.eps_vir.copy(), inp.eps_vir.copy()
        ep[e] += h
        em[e] -= h
        Ep = o.pt2_pass(inp.eps_core, inp.eps_act, ep, inp.gamma_act, inp.B, s, False).E
        Em = o.pt2_pass(inp.eps_core, inp.eps_act, em, inp.gamma_act, inp.B, s, False).E
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - r.D_vv[e, e]) <= 1e-7 * abs(r.D_vv[e, e])


def test_mp2_limit_density_diagonal_fractional_occupations():
    """Same pin with a diagonal, fractional active density (weights n_k n_l)."""
    inp = synth.generate(2, 2, 5, 9, seed=6)
    inp = inp.replace(gamma_act=np.diag([1.4, 0.6]))
    s = 1e5
    r = o.pt2_pass_inputs(inp, s)
    h = 1e-5
    for e in range(inp.n_vir):
        ep, em = inp.eps_vir.copy(), inp.eps_vir.copy()
        ep[e] += h
        em[e] -= h
        Ep = o.pt2_pass(inp.eps_core, inp.eps_act, ep, inp.gamma_act, inp.B, s, False).E
        Em = o.pt2_pass(inp.eps_core, inp.eps_act, em, inp.gamma_act, inp.B, s, False).E
        assert abs((Ep - Em) / (2 * h) - r.D_vv[e, e]) <= 1e-7 * abs(r.D_vv[e, e])


def test_mp2_limit_density_off_diagonal_via_fock_perturbation():
    """Off-diagonal Gamma_ef = 1/2 dE/d(eta) for f_vv = diag(eps) + eta (E_ef + E_fe).
    MP2 is invariant to virtual rotations, so E(eta) is the canonical MP2 energy
    after diagonalizing f_vv and rotating B."""
    inp = _closed(3, 6, 10, seed=8)
    s = 1e3
    r = o.pt2_pass_inputs(inp, s)

    def energy(eta, e, f):
        F = np.diag(inp.eps_vir)
        F[e, f] += eta
        F[f, e] += eta
        w, W = np.linalg.eigh(F)
        Bt = np.einsum("ap,iaQ->ipQ", W, inp.B)
        return o.pt2_pass(inp.eps_core, inp.eps_act, w, inp.gamma_act, Bt, s, False).E

    h = 1e-5
    for e, f in [(0, 1), (1, 4), (2, 5), (3, 3)]:
        fd = (energy(h, e, f) - energy(-h, e, f)) / (2 * h)
        want = 2.0 * r.D_vv[e, f] if e != f else 2.0 * r.D_vv[e, e]
        assert abs(fd - want) <= 1e-6 * np.abs(r.D_vv).max()


# ---------------------------------------------------------------------------
# Small-s closed form: t ~ s V Delta, renormalized V ~ 2 V
# ---------------------------------------------------------------------------

def test_small_s_expansion():
    inp = _closed(3, 5, 8, seed=2)
    eh, ev = inp.eps_core, inp.eps_vir
    lead = 0.0
    for i in range(3):
        for j in range(3):
            V = np.einsum("aQ,bQ->ab", inp.B[i], inp.B[j])
            dl = eh[i] + eh[j] - ev[:, None] - ev[None, :]
            lead += 2.0 * float(np.sum(dl * V * (2 * V - V.T)))
    for s in (1e-4, 1e-5):
        E = o.pt2_pass_inputs(inp, s, with_density=False).E
        assert abs(E / s - lead) <= 50 * s * abs(lead)


# ---------------------------------------------------------------------------
# Invariances and special cases
# ---------------------------------------------------------------------------

def test_aux_rotation_invariance():
    inp = synth.config_inputs("c1")
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((inp.n_aux, inp.n_aux)))
    r0 = o.pt2_pass_inputs(inp, 0.5)
    r1 = o.pt2_pass_inputs(inp.replace(B=inp.B @ Q), 0.5)
    assert abs(r0.E - r1.E) <= 1e-12 * abs(r0.E)
    np.testing.assert_allclose(r1.D_vv, r0.D_vv, atol=1e-12 * np.abs(r0.D_vv).max())


def test_virtual_permutation_equivariance():
    inp = synth.generate(2, 2, 6, 7, seed=9)
    perm = np.array([3, 0, 5, 1, 4, 2])
    r0 = o.pt2_pass_inputs(inp, 0.8)
    r1 = o.pt2_pass_inputs(inp.replace(eps_vir=inp.eps_vir[perm], B=inp.B[:, perm, :]), 0.8)
    assert abs(r0.E - r1.E) <= 1e-13 * abs(r0.E)
    np.testing.assert_allclose(r1.D_vv, r0.D_vv[np.ix_(perm, perm)], atol=1e-14 * np.abs(r0.D_vv).max())


def test_active_rotation_invariance_of_density_contraction():
    """Rotating the active orbitals changes the semicanonical energies' basis, so
    with equal active energies the pass must be invariant to an active rotation
    applied consistently to Gamma_act and B."""
    inp = synth.generate(2, 4, 5, 6, seed=12)
    ea = np.full(4, -0.15)
    inp = inp.replace(eps_act=ea)
    rng = np.random.default_rng(3)
    R, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    B2 = inp.B.copy()
    B2[2:] = np.einsum("uv,uaQ->vaQ", R, inp.B[2:])
    G2 = R.T @ inp.gamma_act @ R
    r0 = o.pt2_pass_inputs(inp, 0.6)
    r1 = o.pt2_pass_inputs(inp.replace(B=B2, gamma_act=G2), 0.6)
    assert abs(r0.E - r1.E) <= 1e-12 * abs(r0.E)
    np.testing.assert_allclose(r1.D_vv, r0.D_vv, atol=1e-12 * np.abs(r0.D_vv).max())


def test_gamma_act_full_occupation_is_closed_shell():
    inp = synth.generate(3, 2, 6, 8, seed=13)
    full = o.pt2_pass_inputs(inp.replace(gamma_act=2.0 * np.eye(2)), 0.5)
    closed = o.pt2_pass(np.concatenate([inp.eps_core, inp.eps_act]), np.zeros(0), inp.eps_vir,
                        np.zeros((0, 0)), inp.B, 0.5)
    assert abs(full.E - closed.E) <= 1e-13 * abs(closed.E)
    np.testing.assert_allclose(full.D_vv, closed.D_vv, atol=1e-13 * np.abs(closed.D_vv).max())


def test_gamma_act_empty_is_core_only():
    inp = synth.generate(3, 2, 6, 8, seed=14)
    empty = o.pt2_pass_inputs(inp.replace(gamma_act=np.zeros((2, 2))), 0.5)
    core = o.pt2_pass(inp.eps_core, np.zeros(0), inp.eps_vir, np.zeros((0, 0)), inp.B[:3], 0.5)
    assert abs(empty.E - core.E) <= 1e-13 * abs(core.E)
    np.testing.assert_allclose(empty.D_vv, core.D_vv, atol=1e-13 * np.abs(core.D_vv).max())


def test_single_pair_closed_form():
    """One doubly occupied hole: D = 2 T T (T symmetric), so ONs = 2 eig(T)^2."""
    inp = _closed(1, 9, 12, seed=5)
    s = 0.9
    r = o.pt2_pass_inputs(inp, s)
    V = np.einsum("aQ,bQ->ab", inp.B[0], inp.B[0])
    dl = 2 * inp.eps_core[0] - inp.eps_vir[:, None] - inp.eps_vir[None, :]
    T = V * (-np.expm1(-s * dl * dl)) / dl
    lam = np.linalg.eigvalsh(T)
    want = np.sort(2.0 * lam ** 2)[::-1]
    occ, _ = o.natural_orbitals(r.D_vv)
    np.testing.assert_allclose(occ, want, rtol=1e-12, atol=1e-15 * want.max())


def test_density_symmetric_psd_and_trace():
    inp = synth.generate(3, 4, 10, 12, seed=21)
    r = o.pt2_pass_inputs(inp, 0.5)
    D = r.D_vv
    assert np.abs(D - D.T).max() <= 1e-15 * np.abs(D).max()
    occ, vecs = o.natural_orbitals(D)
    assert occ.min() > -1e-14 * occ.max()          # Lambda = 0: D is a Gram sum
    assert abs(occ.sum() - np.trace(D)) <= 1e-13 * abs(np.trace(D))
    np.testing.assert_allclose(D @ vecs, vecs * occ[None, :], atol=1e-13 * occ.max())
    np.testing.assert_allclose(vecs.T @ vecs, np.eye(10), atol=1e-13)


def test_density_scales_with_amplitude_square():
    """Scaling B by c scales t by c^2 and D by c^4 (quadratic in t, Eq. A9)."""
    inp = _closed(2, 5, 6, seed=1)
    r1 = o.pt2_pass_inputs(inp, 0.5)
    r2 = o.pt2_pass_inputs(inp.replace(B=inp.B * 1.5), 0.5)
    np.testing.assert_allclose(r2.D_vv, r1.D_vv * 1.5 ** 4, rtol=1e-12, atol=1e-16)
    assert abs(r2.E - r1.E * 1.5 ** 4) <= 1e-12 * abs(r2.E)


# ---------------------------------------------------------------------------
# Truncation (Eqs. 9-10, near-degeneracy rule)
# ---------------------------------------------------------------------------

def test_truncation_hand_made_spectra():
    occ = np.array([4.0, 3.0, 2.0, 1.0])              # cumulative 0.4 0.7 0.9 1.0
    assert o.kept_count_po(occ, 0.7)[0] == 2           # exactly reached -> kept
    assert o.kept_count_po(occ, 0.71)[0] == 3
    assert o.kept_count_po(occ, 1.0)[0] == 4
    assert o.kept_count_po(occ, 0.1)[0] == 1
    n, (below, above) = o.kept_count_po(occ, 0.8)
    assert n == 3 and abs(below - 0.1) < 1e-15 and abs(above - 0.1) < 1e-15
    eq = np.ones(10)
    assert o.kept_count_po(eq, 0.55)[0] == 6
    assert o.kept_count_pv(539, 210 / 539) == 210
    assert o.kept_count_cutoff(occ, 2.0) == 3
    with pytest.raises(ValueError):
        o.kept_count_po(occ, 0.0)


def test_near_degeneracy_expansion():
    occ = np.array([5.0, 2.0, 1.995, 1.985, 1.97, 1.0])
    n, _ = o.kept_count_po(occ, (5.0 + 2.0) / occ.sum())
    assert n == 2
    assert o.expand_near_degenerate(occ, n, 0.0) == 2
    assert o.expand_near_degenerate(occ, n, 0.01) == 4     # anchored at n_last = 2.0
    assert o.expand_near_degenerate(occ, 6, 0.01) == 6


def test_paper_kept_fraction_of_table1():
    """Ni(CO)4, Table 1: N_V' = 210 of 539 retained virtuals at p_o = 98 %, i.e.
    p_v = 38.96 % (Eq. 9); the quartic cost model of Eq. 6 gives (539/210)^4 = 43.4."""
    assert abs(210 / 539 - 0.3896) < 1e-4
    assert abs((539 / 210) ** 4 - 43.4) < 0.05


# ---------------------------------------------------------------------------
# Recanonicalization and the additive correction (Sec. 2, Eq. 11)
# ---------------------------------------------------------------------------

def test_correction_vanishes_without_truncation():
    inp = synth.config_inputs("c1")
    res = o.full_pipeline(inp, 0.5, 1.0)
    assert res["n_kept"] == inp.n_vir
    assert abs(res["correction"][0] + res["correction"][1]) <= 1e-12 * abs(res["energy"][0])


def test_identity_transform_reproduces_energy():
    inp = _closed(4, 8, 9, seed=17)
    E0 = o.pt2_pass_inputs(inp, 0.5, False).energy
    U, et = o.recanonicalize(np.eye(8), inp.eps_vir)
    np.testing.assert_allclose(np.abs(U), np.eye(8), atol=1e-15)
    Bt = o.transform_b(inp.B, U)
    E1 = o.pt2_pass(inp.eps_core, inp.eps_act, et, inp.gamma_act, Bt, 0.5, False).energy
    assert abs(E0[0] - E1[0]) <= 1e-14 * abs(E0[0])


def test_recanonicalized_fock_is_diagonal():
    inp = _closed(2, 10, 5, seed=19)
    r = o.pt2_pass_inputs(inp, 0.5)
    occ, vecs = o.natural_orbitals(r.D_vv)
    U, et = o.recanonicalize(vecs[:, :6], inp.eps_vir)
    F = U.T @ np.diag(inp.eps_vir) @ U
    np.testing.assert_allclose(F, np.diag(et), atol=1e-13)
    np.testing.assert_allclose(U.T @ U, np.eye(6), atol=1e-13)


def _random_orthogonal(n, seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


def _energy_without_recanonicalization(inp, no_kept, s):
    """A wrong kept-space energy for the checks below: B transformed by the kept NOs
    as they are, denominators from the diagonal of F' = V_k^T diag(eps_v) V_k."""
    F = no_kept.T @ (inp.eps_vir[:, None] * no_kept)
    Bt = o.transform_b(inp.B, no_kept)
    return o.pt2_pass(inp.eps_core, inp.eps_act, np.diag(F).copy(), inp.gamma_act, Bt, s, False).energy


@pytest.mark.parametrize("n_act", [0, 2])
def test_kept_energy_depends_only_on_the_kept_space(n_act):
    """Sec. 2 rebuilds the Hamiltonian in the span of the kept NOs and
    recanonicalizes it, so E_kept is a function of that subspace alone: any
    rotation R of the kept NO columns leaves it unchanged.  Skipping the
    recanonicalization (or using diag F') breaks this, and the check shows it."""
    inp = synth.generate(3, n_act, 12, 10, seed=23)
    s, k = 0.5, 7
    occ, vecs = o.natural_orbitals(o.pt2_pass_inputs(inp, s).D_vv)
    R = _random_orthogonal(k, 5)
    e0 = o.kept_energy(inp, vecs, k, s)
    e1 = o.kept_energy(inp, vecs[:, :k] @ R, k, s)
    scale = abs(e0[0])
    assert o.dd_sub(e0, e1)[0] == pytest.approx(0.0, abs=1e-13 * scale)
    w0 = _energy_without_recanonicalization(inp, vecs[:, :k], s)
    w1 = _energy_without_recanonicalization(inp, vecs[:, :k] @ R, s)
    assert abs(o.dd_sub(w0, w1)[0]) > 1e-6 * scale


@pytest.mark.parametrize("n_act,seed", [(0, 29), (2, 31)])
def test_kept_energy_on_canonical_virtual_subset(n_act, seed):
    """When the kept space is spanned by a subset S of the canonical virtuals, the
    recanonicalized basis is that subset (the eps_a are distinct), so E_kept must
    equal the plain pass on the sub-problem (eps_v[S], B[:, S, :]) -- whatever
    rotation within span(S) the kept vectors arrive in."""
    inp = synth.generate(3, n_act, 11, 9, seed=seed)
    s = 0.7
    S = np.sort(np.random.default_rng(seed).choice(inp.n_vir, size=6, replace=False))
    no_kept = np.eye(inp.n_vir)[:, S] @ _random_orthogonal(len(S), seed + 1)
    e_kept = o.kept_energy(inp, no_kept, len(S), s)
    sub = o.pt2_pass(inp.eps_core, inp.eps_act, inp.eps_vir[S], inp.gamma_act,
                     np.ascontiguousarray(inp.B[:, S, :]), s, False).energy
    assert abs(o.dd_sub(e_kept, sub)[0]) <= 1e-13 * abs(sub[0])
    wrong = _energy_without_recanonicalization(inp, no_kept, s)
    assert abs(o.dd_sub(wrong, sub)[0]) > 1e-6 * abs(sub[0])


# ---------------------------------------------------------------------------
# The reading of the input recipe, checked against independently computed values
# ---------------------------------------------------------------------------

def test_c1_reference_values():
    """Values computed when the workload recipe was first specified, by separate
    code; they pin the generator's draw order and the readings, not physics."""
    inp = synth.config_inputs("c1")
    res = o.full_pipeline(inp, 0.5, 0.985)
    assert abs(res["energy"][0] - (-20.267319766453)) < 5e-12
    assert res["n_kept"] == 40
    assert abs(res["margins"][0] - 3.5e-4) < 1e-5 and abs(res["margins"][1] - 9.9e-4) < 1e-5
    e_mp2 = o.pt2_pass_inputs(inp, 1e3, with_density=False).E
    assert abs(e_mp2 - (-20.926912642285)) < 5e-12


def test_double_double_energy():
    parts = [1e8, 1e-9, -1e8, 3e-9]
    hi, lo = o.dd_from_parts(parts)
    assert abs(hi + lo - 4e-9) < 1e-24

"""Second-quantized brute force in a tiny Fock space, used to pin the oracle.

Independent of the oracle's spin-adapted matrix formulas: it builds fermion
operators by the Jordan-Wigner construction over spin orbitals, the reference
ensemble as a quasi-free (zero-cumulant) density operator with a prescribed
spin-summed hole 1-RDM, the first-order doubles operator
    T = sum_{I<J, A<B} t^{IJ}_{AB} a+_A a+_B a_J a_I,
    t^{IJ}_{AB} = <AB||IJ> (1 - e^{-s Delta^2}) / Delta           (App. A, Eq. A7)
with antisymmetrized spin-orbital integrals, A = T - T^+, and then evaluates
    Gamma^(2)_ef = 1/2 Tr( rho [[E_ef, A], A] ),  E_ef = sum_sigma a+_{e sigma} a_{f sigma}
        (App. A, Eq. A8: the doubly nested commutator of the virtual block)
    E^(2)        = Tr( rho [V, A] ) + 1/2 Tr( rho [[H0, A], A] )
        (App. A, Eq. A4: the scalar part of the second-order Hamiltonian)
as plain matrix traces.  For a quasi-free rho every normal-ordered remainder has
zero expectation, so the traces are the fully contracted scalars of the paper.

With ``B_act`` (integrals B^Q_ix of hole i and active particle x) the particle
indices of the doubles run over active and virtual orbitals, as in the
multireference theory (holes: core and active; particles: active and virtual;
excitations with four active indices are internal and left out).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _jw_annihilators(n_modes: int):
    lower = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
    z = sp.csr_matrix(np.diag([1.0, -1.0]))
    eye = sp.identity(2, format="csr")
    ops = []
    for k in range(n_modes):
        m = sp.identity(1, format="csr")
        for q in range(n_modes):
            f = z if q < k else (lower if q == k else eye)
            m = sp.kron(m, f, format="csr")
        ops.append(m)
    return ops


def _occupation_probabilities(n_modes, probs):
    """Diagonal of a product density operator; mode k occupied with probs[k]."""
    diag = np.ones(1)
    for k in range(n_modes):
        p = probs[k]
        diag = np.kron(diag, np.array([1.0 - p, p]))
    return diag


def singlet_pair_states(n_act, coeffs):
    """Two-electron singlet states of the active orbitals in their own Jordan-Wigner
    space (2 n_act modes, spin orbital 2 u + sigma): psi = sum_uv C_uv a+_{u up} a+_{v dn} |0>
    with C symmetric (a singlet) and normalized.  coeffs: list of symmetric C."""
    c = _jw_annihilators(2 * n_act)
    vac = np.zeros(2 ** (2 * n_act))
    vac[0] = 1.0
    out = []
    for C in coeffs:
        C = 0.5 * (C + C.T)
        psi = np.zeros_like(vac)
        for u in range(n_act):
            for v in range(n_act):
                psi += C[u, v] * (c[2 * u].T @ (c[2 * v + 1].T @ vac))
        out.append(psi / np.linalg.norm(psi))
    return out


def active_rdms(n_act, weights, states):
    """Spin-free active 1-RDM gamma_u^v, 2-cumulant lambda_uv^xy and 3-cumulant
    lambda_uvw^xyz of the ensemble sum_a w_a |psi_a><psi_a| (states from
    singlet_pair_states).  Spin-orbital cumulants by the usual subtraction of
    antisymmetrized products, spin-free ones as sums over matching spins."""
    n = 2 * n_act
    c = [x.toarray() for x in _jw_annihilators(n)]
    cd = [x.T for x in c]

    def ev(op):
        return sum(w * psi @ (op @ psi) for w, psi in zip(weights, states))

    g1 = np.array([[ev(cd[p] @ c[q]) for q in range(n)] for p in range(n)])
    g2 = np.zeros((n,) * 4)
    for p in range(n):
        for q in range(n):
            pq = cd[p] @ cd[q]
            for r in range(n):
                for t in range(n):
                    g2[p, q, r, t] = ev(pq @ c[t] @ c[r])   # <a+_p a+_q a_t a_r> = gamma^pq_rt
    g3 = np.zeros((n,) * 6)
    for p in range(n):
        for q in range(n):
            for r in range(n):
                pqr = cd[p] @ cd[q] @ cd[r]
                if not np.any(pqr):
                    continue
                for x in range(n):
                    for y in range(n):
                        for z in range(n):
                            g3[p, q, r, x, y, z] = ev(pqr @ c[z] @ c[y] @ c[x])
    l2 = g2 - np.einsum("pr,qs->pqrs", g1, g1) + np.einsum("ps,qr->pqrs", g1, g1)
    # gamma3 = l3 + A(g1 l2) + A(g1 g1 g1): all ways of giving one upper and one lower
    # index to a factor, with the sign of the permutation of the lower indices
    import itertools
    perms = list(itertools.permutations(range(3)))

    def sign(pm):
        s_, pm = 1, list(pm)
        for i in range(3):
            for j in range(i + 1, 3):
                if pm[i] > pm[j]:
                    s_ = -s_
        return s_

    up = "pqr"
    lo = "xyz"
    a1l2 = np.zeros_like(g3)
    a111 = np.zeros_like(g3)
    for pm in perms:
        sg = sign(pm)
        lw = "".join(lo[k] for k in pm)     # lower index given to each upper position
        a111 += sg * np.einsum(f"{up[0]}{lw[0]},{up[1]}{lw[1]},{up[2]}{lw[2]}->pqrxyz", g1, g1, g1)
        # one upper index (position i) with its lower partner in g1, the other two in l2
        for i in range(3):
            rest = [k for k in range(3) if k != i]
            a1l2 += sg * np.einsum(f"{up[i]}{lw[i]},{up[rest[0]]}{up[rest[1]]}{lw[rest[0]]}{lw[rest[1]]}->pqrxyz",
                                   g1, l2) / 2.0
    l3 = g3 - a1l2 - a111
    # spin-free sums over matching spins (spin orbital 2 u + sigma)
    G = g1.reshape(n_act, 2, n_act, 2)
    gamma = np.einsum("usvs->uv", G)
    L2 = l2.reshape(n_act, 2, n_act, 2, n_act, 2, n_act, 2)
    lam2 = np.einsum("asbtcsdt->abcd", L2)
    L3 = l3.reshape((n_act, 2) * 6)
    lam3 = np.einsum("asbtcrdsetfr->abcdef", L3)
    return gamma, lam2, lam3, dict(g1=g1, g2=g2, g3=g3, l2=l2, l3=l3)


def brute_force_pt2(eps_core, eps_act, eps_vir, gamma_act, B, s, B_act=None, states=None, singles=None,
                    probe_singles_source=False):
    """Return (E2, Gamma_vv, gamma_act) by explicit Fock-space traces.

    Spatial orbitals: core, active, virtual.  Spin orbital index 2 p + sigma.
    B_act [n_h, n_act, n_aux]: with it, active particle indices are included.
    states: None for the quasi-free reference with active 1-RDM gamma_act, or
    (weights, vectors) of a correlated ensemble over the active orbitals (vectors in
    the active orbitals' own Jordan-Wigner space, singlet_pair_states), the core
    doubly occupied and the virtuals empty; gamma_act is then ignored.
    singles: None, or t1[i, e] = t_e^i, spin-free singles amplitudes of hole i and
    virtual e added to the cluster operator as sum_sigma t_e^i a+_{e sigma} a_{i sigma}.
    probe_singles_source (quasi-free reference only): instead, return src[i, e, sigma],
    the coefficient of {a+_{e sigma} a_{i sigma}} in the one-body part of [H0, T2]
    (the first-order source of the singles), read off the generalized Wick theorem:
    for a quasi-free reference <{a+_i a_e} X> = sum_q gamma^i_q X^e_q, since a one-body
    normal-ordered string cannot fully contract with a two-body one; core holes have
    gamma^m_q = delta_mq, active holes are solved for with the active 1-RDM."""
    n_c, n_a, n_v = len(eps_core), len(eps_act), len(eps_vir)
    n_h = n_c + n_a
    n_sp = n_h + n_v
    n_modes = 2 * n_sp
    eps = np.concatenate([eps_core, eps_act, eps_vir])
    c = _jw_annihilators(n_modes)

    if states is None:
        # natural orbitals of the active block: Gamma_act = U diag(n) U^T
        if n_a:
            occ_nat, U = np.linalg.eigh(gamma_act)
        else:
            occ_nat, U = np.zeros(0), np.zeros((0, 0))
        # c_k: annihilators of natural spin orbitals (Jordan-Wigner modes)
        probs = np.zeros(n_modes)
        for p in range(n_c):
            probs[2 * p] = probs[2 * p + 1] = 1.0
        for k in range(n_a):
            probs[2 * (n_c + k)] = probs[2 * (n_c + k) + 1] = occ_nat[k] / 2.0
        rho = sp.diags(_occupation_probabilities(n_modes, probs), format="csr")

        # semicanonical annihilators: a_(u sigma) = sum_k U_uk c_(k sigma)
        a = list(c)
        for ui in range(n_a):
            for sig in range(2):
                op = None
                for k in range(n_a):
                    term = U[ui, k] * c[2 * (n_c + k) + sig]
                    op = term if op is None else op + term
                a[2 * (n_c + ui) + sig] = op.tocsr()

        def tr(x):
            return float((rho @ x).diagonal().sum())
    else:
        # |core filled> (x) |psi_active> (x) |virtuals empty> in the full Jordan-Wigner basis
        weights, vecs = states
        core = np.zeros(2 ** (2 * n_c))
        core[-1] = 1.0
        virt = np.zeros(2 ** (2 * n_v))
        virt[0] = 1.0
        full = [np.kron(np.kron(core, v), virt) for v in vecs]
        a = list(c)

        def tr(x):
            return float(sum(w * f @ (x @ f) for w, f in zip(weights, full)))
    ad = [x.T.tocsr() for x in a]

    # spatial integrals (ai|bj) = sum_Q B^Q_ia B^Q_jb, written with explicit indices
    Vsp = np.einsum("iaQ,jbQ->ijab", B, B)

    holes = [(i, sig) for i in range(n_h) for sig in range(2)]
    virts = [(n_h + a_, sig) for a_ in range(n_v) for sig in range(2)]
    if B_act is not None:
        # particles: active then virtual; B_all[i, p] over particle orbitals p
        virts = [(n_c + x_, sig) for x_ in range(n_a) for sig in range(2)] + virts
        B_all = np.concatenate([B_act, B], axis=1)
        Vall = np.einsum("ipQ,jqQ->ijpq", B_all, B_all)

    def so(p):
        return 2 * p[0] + p[1]

    def g(A_, B_, I_, J_):
        """<AB|IJ> in spin orbitals (physicists' notation; spin-free part (ai|bj))."""
        if A_[1] != I_[1] or B_[1] != J_[1]:
            return 0.0
        if B_act is None:
            return Vsp[I_[0], J_[0], A_[0] - n_h, B_[0] - n_h]
        return Vall[I_[0], J_[0], A_[0] - n_c, B_[0] - n_c]

    def internal(*idx):
        return all(n_c <= q[0] < n_h for q in idx)

    # one-body contractions c(p, q) = Tr(rho a+_p a_q) of the reference, for the
    # normal-ordered excitation operators of the cluster operator
    cmat = {}

    def cval(p, q):
        key = (so(p), so(q))
        if key not in cmat:
            cmat[key] = tr(ad[key[0]] @ a[key[1]])
        return cmat[key]

    def excitation(A_, B_, I_, J_):
        """{a+_A a+_B a_J a_I}: normal ordered with respect to the (quasi-free)
        reference, i.e. the bare product minus its contractions (Wick)."""
        ex = ad[so(A_)] @ ad[so(B_)] @ a[so(J_)] @ a[so(I_)]
        cAI, cAJ, cBI, cBJ = cval(A_, I_), cval(A_, J_), cval(B_, I_), cval(B_, J_)
        if cAI or cAJ or cBI or cBJ:
            one = sp.identity(ex.shape[0], format="csr")
            ex = (ex - cAI * (ad[so(B_)] @ a[so(J_)]) + cAJ * (ad[so(B_)] @ a[so(I_)])
                  - cBJ * (ad[so(A_)] @ a[so(I_)]) + cBI * (ad[so(A_)] @ a[so(J_)])
                  + (cAI * cBJ - cAJ * cBI) * one)
        return ex.tocsr()

    T = None
    Vop = None
    for x in range(len(holes)):
        for y in range(x + 1, len(holes)):
            I_, J_ = holes[x], holes[y]
            for p in range(len(virts)):
                for q in range(p + 1, len(virts)):
                    A_, B_ = virts[p], virts[q]
                    if internal(I_, J_, A_, B_):
                        continue
                    v = g(A_, B_, I_, J_) - g(A_, B_, J_, I_)
                    if v == 0.0:
                        continue
                    dl = eps[I_[0]] + eps[J_[0]] - eps[A_[0]] - eps[B_[0]]
                    t = v * (1.0 - np.exp(-s * dl * dl)) / dl
                    ex = excitation(A_, B_, I_, J_)
                    T = t * ex if T is None else T + t * ex
                    Vop = v * ex if Vop is None else Vop + v * ex
    if probe_singles_source:
        assert states is None and singles is None
        H0p = None
        for p_ in range(n_sp):
            for sig in range(2):
                k = 2 * p_ + sig
                term = eps[p_] * (ad[k] @ a[k])
                H0p = term if H0p is None else H0p + term
        X = (H0p @ T - T @ H0p).tocsr()
        src = np.zeros((n_h, n_v, 2))
        ga = gamma_act / 2.0                                 # per-spin active 1-RDM
        for e_ in range(n_v):
            for sig in range(2):
                ke = 2 * (n_h + e_) + sig
                probe = [tr(ad[2 * i_ + sig] @ a[ke] @ X) for i_ in range(n_h)]
                src[:n_c, e_, sig] = probe[:n_c]
                if n_a:
                    src[n_c:, e_, sig] = np.linalg.solve(ga, np.array(probe[n_c:]))
        return src
    if singles is not None:
        for i_ in range(n_h):
            for e_ in range(n_v):
                if singles[i_, e_] == 0.0:
                    continue
                for sig in range(2):
                    ex = ad[2 * (n_h + e_) + sig] @ a[2 * i_ + sig]     # {a+_e a_i}: gamma^e_i = 0
                    T = singles[i_, e_] * ex if T is None else T + singles[i_, e_] * ex
    Aop = (T - T.T).tocsr()
    Vop = (Vop + Vop.T).tocsr()
    H0 = None
    for p in range(n_sp):
        for sig in range(2):
            k = 2 * p + sig
            term = eps[p] * (ad[k] @ a[k])
            H0 = term if H0 is None else H0 + term

    def comm(x, y):
        return (x @ y - y @ x).tocsr()

    E2 = tr(comm(Vop, Aop)) + 0.5 * tr(comm(comm(H0, Aop), Aop))
    Gvv = np.zeros((n_v, n_v))
    for e in range(n_v):
        for f in range(n_v):
            Eef = None
            for sig in range(2):
                term = ad[2 * (n_h + e) + sig] @ a[2 * (n_h + f) + sig]
                Eef = term if Eef is None else Eef + term
            Gvv[e, f] = 0.5 * tr(comm(comm(Eef, Aop), Aop))
    # sanity of the reference: the active 1-RDM it carries
    gam = np.zeros((n_a, n_a))
    for ui in range(n_a):
        for vi in range(n_a):
            gam[ui, vi] = sum(tr(ad[2 * (n_c + ui) + sg] @ a[2 * (n_c + vi) + sg]) for sg in range(2))
    return E2, Gvv, gam

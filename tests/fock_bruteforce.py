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


def brute_force_pt2(eps_core, eps_act, eps_vir, gamma_act, B, s, B_act=None):
    """Return (E2, Gamma_vv) by explicit Fock-space traces.

    Spatial orbitals: core, active, virtual.  Spin orbital index 2 p + sigma.
    B_act [n_h, n_act, n_aux]: with it, active particle indices are included."""
    n_c, n_a, n_v = len(eps_core), len(eps_act), len(eps_vir)
    n_h = n_c + n_a
    n_sp = n_h + n_v
    n_modes = 2 * n_sp
    eps = np.concatenate([eps_core, eps_act, eps_vir])

    # natural orbitals of the active block: Gamma_act = U diag(n) U^T
    if n_a:
        occ_nat, U = np.linalg.eigh(gamma_act)
    else:
        occ_nat, U = np.zeros(0), np.zeros((0, 0))
    # c_k: annihilators of natural spin orbitals (Jordan-Wigner modes)
    c = _jw_annihilators(n_modes)
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
    ad = [x.T.tocsr() for x in a]

    def tr(x):
        return float((rho @ x).diagonal().sum())

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

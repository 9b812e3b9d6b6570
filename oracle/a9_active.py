"""Eq. A9 terms with an active particle index, at zero density cumulants.

TEST INFRASTRUCTURE ONLY (see the package docstring).

In the multireference theory the particle indices of the first-order doubles run
over active and virtual orbitals (Eq. A7; holes i, j are core or active).  The
virtual block of the second-order 1-RDM (Eq. A9) then has, besides the three
terms with two virtual particle indices (oracle.dsrg_pt2), terms whose
amplitudes carry one virtual and one active particle index.  With zero
cumulants (Lambda_2 = Lambda_3 = 0) and without singles they are
    t^{ev}_{mn} tc^{fu}_{mn} eta^u_v                                 (core-core holes)
  + 1/2 S( t^{ey}_{mu} tc^{fx}_{mv} ) Gamma^u_v eta^x_y              (core-active holes)
  + 1/4 t^{ez}_{ux} tc^{fw}_{vy} Gamma^u_v Gamma^x_y eta^w_z         (active-active holes)
with eta = 2 - Gamma (the spin-summed active hole density), the exchange
combination tc^{ab}_{ij} = 2 t^{ab}_{ij} - t^{ab}_{ji}, and S() adding the term
with both amplitudes' hole indices swapped.  Amplitudes (Eq. A7):
    t^{ex}_{ij} = <ex|ij> (1 - e^{-s Delta^2}) / Delta,
    <ex|ij> = sum_Q B^Q_ie B^Q_jx,   Delta = eps_i + eps_j - eps_e - eps_x,
with B^Q_jx the density-fitted integrals of hole j and active particle x.
For an ordered hole pair (i, j) the n_v x n_act matrix X_ij holds t^{ex}_{ij}.

Reading: the paper prints the active-active term with a plain t on the second
amplitude; a Fock-space evaluation of 1/2 <[[E_ef, A], A]> over a quasi-free
reference (tests/fock_bruteforce.py) fixes it as the exchange combination tc,
i.e. 1/2 t t eta (Gamma^u_v Gamma^x_y - 1/2 Gamma^x_v Gamma^u_y), the same
zero-cumulant 2-RDM that weights the active-active term with virtual particles.
"""
from __future__ import annotations

import numpy as np


def active_particle_amplitudes(eps_h, eps_act, eps_vir, B, B_act, i, j, s):
    """X_ij [e, x] = t^{ex}_{ij} (Eq. A7 with particle indices e virtual, x active)."""
    V = B[i] @ B_act[j].T
    dl = eps_h[i] + eps_h[j] - eps_vir[:, None] - eps_act[None, :]
    return V * (1.0 - np.exp(-s * dl * dl)) / dl


def active_particle_density(eps_core, eps_act, eps_vir, gamma_act, B, B_act, s):
    """The three zero-cumulant Eq. A9 terms above, spin-summed, [n_v, n_v]."""
    n_core, n_act, n_v = len(eps_core), len(eps_act), len(eps_vir)
    n_h = n_core + n_act
    eps_h = np.concatenate([eps_core, eps_act])
    G = gamma_act
    eta = 2.0 * np.eye(n_act) - G
    X = {(i, j): active_particle_amplitudes(eps_h, eps_act, eps_vir, B, B_act, i, j, s)
         for i in range(n_h) for j in range(n_h)}

    def Xc(i, j):
        return 2.0 * X[i, j] - X[j, i]

    core = range(n_core)
    act = range(n_core, n_h)
    D = np.zeros((n_v, n_v))
    for m in core:
        for n in core:
            D += X[m, n] @ eta @ Xc(m, n).T
    for m in core:
        for ui, u in enumerate(act):
            for vi, v in enumerate(act):
                D += 0.5 * G[ui, vi] * (X[m, u] @ eta @ Xc(m, v).T + X[u, m] @ eta @ Xc(v, m).T)
    for ui, u in enumerate(act):
        for xi, x in enumerate(act):
            for vi, v in enumerate(act):
                for yi, y in enumerate(act):
                    D += 0.25 * G[ui, vi] * G[xi, yi] * (X[u, x] @ eta @ Xc(v, y).T)
    return D

"""Singles (Eq. A6) and the density-cumulant terms of Eq. A9.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Index conventions of App. A: a spin-free operator E_p^q = sum_sigma a+_{p sigma}
a_{q sigma} has its creation index first (lower) and its annihilation index
second (upper).  Accordingly
    gamma_u^v        = <E_u^v>                              (Gamma_act[u, v])
    lambda_uv^xy     spin-free 2-cumulant of <a+_u a+_v a_y a_x> (lam[u, v, x, y]),
                     lambda_uv^xy = gamma_uv^xy - gamma_u^x gamma_v^y + 1/2 gamma_u^y gamma_v^x
    t_ab^ij          amplitude of a+_a a+_b a_j a_i (particles a, b; holes i, j)
    t_a^i            amplitude of a+_a a_i
    eta_u^v          = 2 delta_uv - gamma_u^v
Holes i, j run over core (m, n) and active (u, v, w, x, y, z) orbitals, particles
over active and virtual (e, f, e') orbitals.  Denominators
Delta_ab^ij = eps_i + eps_j - eps_a - eps_b and Delta_a^i = eps_i - eps_a.

First-order singles (Eq. A6) with the semicanonical model's f_a^i = 0:
    t_e^i = 1/2 sum_ux Delta_u^x gamma_x^u tc_ex^iu (1 - e^{-s (Delta_e^i)^2}) / Delta_e^i,
    tc_ab^ij = 2 t_ab^ij - t_ab^ji,   Delta_u^x = eps_x - eps_u.
Only singles with a virtual particle enter Gamma_vv.

Terms of Eq. A9 computed here (the others are in oracle.dsrg_pt2 and
oracle.a9_active; the three-body-cumulant term is dropped, Sec. 2):
    D1  2 t_e^m t_f^m + t_e^u t_f^v gamma_u^v                         (singles)
    D2  (t_e^u t_fv^xy + t_ey^uv t_f^x) lambda_uv^xy                  (singles x doubles)
    D3  t_ee'^uv t_fe'^xy lambda_uv^xy                                (the cumulant part of
                                                                       Gamma_uv^xy in the
                                                                       active-active term)
    D4  P( t_ey^mv t_fu^mx ) lambda_uv^xy
    D5  1/2 t_ez^uv t_fw^xy eta_w^z lambda_uv^xy
    D6  1/2 P( t_ey^wv t_fu^zx ) gamma_w^z lambda_uv^xy
with the shorthand P read positionally from its printed definition:
    P( t_{a p}^{i j} t_{c d}^{k q} ) = 2 t_{ap}^{ij} t_{cd}^{kq} - t_{ap}^{ij} t_{cd}^{qk}
                                     - t_{ap}^{ji} t_{cd}^{kq} - t_{aq}^{ji} t_{cd}^{pk},
p the second particle index of the first amplitude and q the second hole index of
the second (the last term trades them).
"""
from __future__ import annotations

import numpy as np


def _amplitude_blocks(eps_h, eps_act, eps_vir, B, B_act, s):
    """X[i, j, e, x] = t_ex^ij (particle e virtual, x active) and
    Tv[u, v, e, f] = t_ef^uv for active holes u, v (Eq. A7, DF integrals)."""
    n_h, n_v, n_aux = B.shape
    n_act = B_act.shape[1]
    n_core = n_h - n_act
    V = np.einsum("ieQ,jxQ->ijex", B, B_act)
    dl = (eps_h[:, None, None, None] + eps_h[None, :, None, None]
          - eps_vir[None, None, :, None] - eps_act[None, None, None, :])
    X = V * (1.0 - np.exp(-s * dl * dl)) / dl
    Ba = B[n_core:]
    Vv = np.einsum("ueQ,vfQ->uvef", Ba, Ba)
    ea = eps_h[n_core:]
    dv = ea[:, None, None, None] + ea[None, :, None, None] - eps_vir[None, None, :, None] - eps_vir[None, None, None, :]
    Tv = Vv * (1.0 - np.exp(-s * dv * dv)) / dv
    return X, Tv


def singles_source(eps_core, eps_act, eps_vir, gamma_act, B, B_act, s):
    """The bracket of Eq. A6 with f = 0: src[i, e] = 1/2 sum_ux Delta_u^x gamma_x^u tc_ex^iu."""
    eps_h = np.concatenate([eps_core, eps_act])
    n_core = len(eps_core)
    X, _ = _amplitude_blocks(eps_h, eps_act, eps_vir, B, B_act, s)
    Xa = X[:, n_core:]                               # t_ex^iu, hole u active: [i, u, e, x]
    Xa_sw = X[n_core:, :].transpose(1, 0, 2, 3)      # t_ex^ui:                 [i, u, e, x]
    tc = 2.0 * Xa - Xa_sw
    dux = eps_act[None, :] - eps_act[:, None]        # Delta_u^x = eps_x - eps_u  [u, x]
    w = dux * gamma_act.T                            # Delta_u^x gamma_x^u        [u, x]
    return 0.5 * np.einsum("ux,iuex->ie", w, tc)


def singles_amplitudes(eps_core, eps_act, eps_vir, gamma_act, B, B_act, s):
    """t[i, e] = t_e^i (Eq. A6, f = 0)."""
    eps_h = np.concatenate([eps_core, eps_act])
    src = singles_source(eps_core, eps_act, eps_vir, gamma_act, B, B_act, s)
    dl = eps_h[:, None] - eps_vir[None, :]
    return src * (1.0 - np.exp(-s * dl * dl)) / dl


def cumulant_singles_density(eps_core, eps_act, eps_vir, gamma_act, lam, B, B_act, s, terms=None):
    """D1 .. D6 above, spin-summed, [n_v, n_v].  lam[u, v, x, y] = lambda_uv^xy.
    `terms` (a subset of {1..6}) selects terms for the checks; default all."""
    terms = set(range(1, 7)) if terms is None else set(terms)
    n_core, n_act, n_v = len(eps_core), len(eps_act), len(eps_vir)
    eps_h = np.concatenate([eps_core, eps_act])
    G = gamma_act
    eta = 2.0 * np.eye(n_act) - G
    X, Tv = _amplitude_blocks(eps_h, eps_act, eps_vir, B, B_act, s)
    t1 = singles_amplitudes(eps_core, eps_act, eps_vir, gamma_act, B, B_act, s)   # [i, e]
    tm, tu = t1[:n_core], t1[n_core:]
    Xaa = X[n_core:, n_core:]          # t_ex^uv with active holes u, v: [u, v, e, x]
    Xca = X[:n_core, n_core:]          # t_ex^mu: [m, u, e, x]
    Xac = X[n_core:, :n_core]          # t_ex^um: [u, m, e, x]
    D = np.zeros((n_v, n_v))
    if 1 in terms:
        D += 2.0 * tm.T @ tm + tu.T @ G @ tu
    if 2 in terms:
        # t_e^u t_fv^xy lambda_uv^xy + t_ey^uv t_f^x lambda_uv^xy
        W1 = np.einsum("xyfv,uvxy->fu", Xaa, lam)
        W2 = np.einsum("uvey,uvxy->ex", Xaa, lam)
        D += tu.T @ W1.T + W2 @ tu
    if 3 in terms:
        D += np.einsum("uvea,xyfa,uvxy->ef", Tv, Tv, lam, optimize=True)
    if 4 in terms:
        # P( t_ey^mv t_fu^mx ) lambda_uv^xy over core m, with (p, q) = (y, x):
        # 2 t_ey^mv t_fu^mx - t_ey^mv t_fu^xm - t_ey^vm t_fu^mx - t_ex^vm t_fu^ym
        for m in range(n_core):
            a_mv, a_vm = Xca[m], Xac[:, m]          # [v, e, y] = t_ey^mv and t_ey^vm
            D += 2.0 * np.einsum("vey,xfu,uvxy->ef", a_mv, a_mv, lam, optimize=True)
            D -= np.einsum("vey,xfu,uvxy->ef", a_mv, a_vm, lam, optimize=True)
            D -= np.einsum("vey,xfu,uvxy->ef", a_vm, a_mv, lam, optimize=True)
            D -= np.einsum("vex,yfu,uvxy->ef", a_vm, a_vm, lam, optimize=True)
    if 5 in terms:
        D += 0.5 * np.einsum("uvez,xyfw,wz,uvxy->ef", Xaa, Xaa, eta, lam, optimize=True)
    if 6 in terms:
        # 1/2 P( t_ey^wv t_fu^zx ) gamma_w^z lambda_uv^xy, all holes active:
        # 2 t_ey^wv t_fu^zx - t_ey^wv t_fu^xz - t_ey^vw t_fu^zx - t_ex^vw t_fu^yz
        D += 0.5 * (2.0 * np.einsum("wvey,zxfu,wz,uvxy->ef", Xaa, Xaa, G, lam, optimize=True)
                    - np.einsum("wvey,xzfu,wz,uvxy->ef", Xaa, Xaa, G, lam, optimize=True)
                    - np.einsum("vwey,zxfu,wz,uvxy->ef", Xaa, Xaa, G, lam, optimize=True)
                    - np.einsum("vwex,yzfu,wz,uvxy->ef", Xaa, Xaa, G, lam, optimize=True))
    return D


def three_cumulant_term(eps_core, eps_act, eps_vir, B, B_act, lam3, s):
    """The term the method drops (Sec. 2), for checks only:
    t_ez^uw t_fv^xy lambda_xyz^uvw, lam3[x, y, z, u, v, w] = lambda_xyz^uvw."""
    eps_h = np.concatenate([eps_core, eps_act])
    n_core = len(eps_core)
    X, _ = _amplitude_blocks(eps_h, eps_act, eps_vir, B, B_act, s)
    Xaa = X[n_core:, n_core:]
    return np.einsum("uwez,xyfv,xyzuvw->ef", Xaa, Xaa, lam3, optimize=True)

"""Plain FP64 reference of the DF-DSRG-PT2 virtual natural-orbital pass.

TEST INFRASTRUCTURE ONLY (see the package docstring).  NumPy in float64; BLAS
matrix products and LAPACK ``eigh`` serve as library steps.  Written for a
reader holding the paper: every function cites the passage it follows.

Notation (paper App. A): core holes m, n; active holes u, v, w, x, y, z;
virtuals e, f, e' (here a, b, c).  Generic holes i, j, k, l run over core then
active.  For an ordered hole pair (i, j) the first-order doubles are the
n_v x n_v matrix T_ij with (T_ij)_ab = t^{ij}_{ab}; the exchange-combined
amplitude is tcheck^{ij}_{ab} = 2 t^{ij}_{ab} - t^{ji}_{ab} = 2 t^{ij}_{ab} - t^{ij}_{ba},
i.e. Tc_ij = 2 T_ij - T_ij^T.

Readings where the paper is silent (each one is listed in the design notes):
  * The DSRG-PT2 energy is not printed in the paper.  We use the spin-adapted
    second-order scalar with renormalized integrals Vr = V (1 + e^{-s D^2}):
        E = 1/4 sum_{ijkl} gamma_ik gamma_jl <Vr_ij, Tc_kl>,
    gamma = 2 I_core (+) Gamma_act (spin-summed hole density, Eq. A1), which is
    what the Wick contraction of [V, A] + 1/2 [[H0, A], A] gives for a
    reference with zero cumulants.  Closed shell: E = sum_ij <Vr_ij, Tc_ij>.
  * Only virtual particle indices enter the amplitudes; Fock off-diagonal
    blocks (singles) are zero; the density cumulants Lambda_2 and Lambda_3 are
    zero.  The virtual 1-RDM is then the three Eq. A9 terms that carry two
    virtual particle indices on both amplitudes (the core-core term, the
    core-active S() term and the active-active term with the reference 2-RDM).
  * The density is spin-summed (the E^p_q of Eq. A1 sums both spins).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# double-double helpers for energies (the sums reach 1e8 Eh while the target
# accuracy is 1e-8 Eh, below one FP64 ulp of the total)
# ----------------------------------------------------------------------------


def dd_from_parts(parts) -> Tuple[float, float]:
    """Correctly rounded sum of the parts as (hi, lo) with hi + lo exact to ~2^-106."""
    parts = list(parts)
    hi = math.fsum(parts)
    lo = math.fsum(parts + [-hi])
    return hi, lo


def dd_sub(a: Tuple[float, float], b: Tuple[float, float]) -> Tuple[float, float]:
    return dd_from_parts([a[0], a[1], -b[0], -b[1]])


# ----------------------------------------------------------------------------
# Building blocks (App. A, Eq. A7 and the text after it)
# ----------------------------------------------------------------------------


def hole_density(n_core: int, gamma_act: np.ndarray) -> np.ndarray:
    """Spin-summed hole 1-RDM gamma = 2 I_core (+) Gamma_act (Eq. A1)."""
    n_act = gamma_act.shape[0]
    g = np.zeros((n_core + n_act, n_core + n_act))
    g[:n_core, :n_core] = 2.0 * np.eye(n_core)
    g[n_core:, n_core:] = gamma_act
    return g


def pair_integrals(B: np.ndarray, i: int, j: int) -> np.ndarray:
    """<ab|ij> in density-fitted form, V^{ij}_{ab} = sum_Q B^Q_ia B^Q_jb (Sec. 3, Eq. A7).

    ``B`` has layout [hole, virtual, aux]."""
    return B[i] @ B[j].T


def pair_denominators(eps_h: np.ndarray, eps_v: np.ndarray, i: int, j: int) -> np.ndarray:
    """Delta^{ij}_{ab} = eps_i + eps_j - eps_a - eps_b (definition after Eq. A7)."""
    return eps_h[i] + eps_h[j] - eps_v[:, None] - eps_v[None, :]


def first_order_doubles(V: np.ndarray, delta: np.ndarray, s: float) -> np.ndarray:
    """t^{ij}_{ab} = <ab|ij> (1 - e^{-s Delta^2}) / Delta (Eq. A7)."""
    return V * (1.0 - np.exp(-s * delta * delta)) / delta


def renormalized_integrals(V: np.ndarray, delta: np.ndarray, s: float) -> np.ndarray:
    """Second-order renormalized integrals V (1 + e^{-s Delta^2}) (energy reading above)."""
    return V * (1.0 + np.exp(-s * delta * delta))


def tcheck(T: np.ndarray) -> np.ndarray:
    """Exchange-combined amplitudes 2 t^{ij}_{ab} - t^{ji}_{ab} (after Eq. A7)."""
    return 2.0 * T - T.T


# ----------------------------------------------------------------------------
# The pass: PT2 energy and the virtual block of the second-order 1-RDM
# ----------------------------------------------------------------------------


@dataclass
class PassResult:
    energy: Tuple[float, float]                 # (hi, lo)
    D_vv: Optional[np.ndarray]                  # [n_v, n_v] spin-summed, or None
    pair_energy: np.ndarray                     # [n_h, n_h] <Vr_ij, Tc_ij>, NaN if not core-core
    pair_tnorm: np.ndarray                      # [n_h, n_h] ||T_ij||_F
    extra: Dict = field(default_factory=dict)

    @property
    def E(self) -> float:
        return self.energy[0] + self.energy[1]


def pt2_pass(eps_core: np.ndarray, eps_act: np.ndarray, eps_vir: np.ndarray,
             gamma_act: np.ndarray, B: np.ndarray, s: float,
             with_density: bool = True, pair_mask: Optional[np.ndarray] = None) -> PassResult:
    """Energy and Gamma^(2)_vv of DF-DSRG-PT2 (Eq. 7, App. A Eqs. A7 and A9).

    Gamma^(2)_ef =  2 t^{mn}_{ee'} tc^{mn}_{fe'}                       (core-core)
                 +  S( t^{mu}_{ee'} tc^{mv}_{fe'} ) Gamma^u_v           (core-active)
                 +  t^{uv}_{ee'} t^{xy}_{fe'} Gamma^{uv}_{xy}           (active-active)
    with S(A^{pq} B^{rs}) = A^{pq} B^{rs} + A^{qp} B^{sr} and, for zero cumulant,
    Gamma^{uv}_{xy} = Gamma^u_x Gamma^v_y - 1/2 Gamma^v_x Gamma^u_y.

    ``pair_mask`` (n_h x n_h, symmetric) drops core-core pairs whose entry is 0
    from both sums; pairs with an active hole are always kept.
    """
    n_core, n_act, n_v = eps_core.shape[0], eps_act.shape[0], eps_vir.shape[0]
    n_h = n_core + n_act
    assert B.shape[:2] == (n_h, n_v)
    eps_h = np.concatenate([eps_core, eps_act])
    G = gamma_act
    core = list(range(n_core))
    act = list(range(n_core, n_h))

    def amps(i, j):
        V = pair_integrals(B, i, j)
        dl = pair_denominators(eps_h, eps_vir, i, j)
        return first_order_doubles(V, dl, s), renormalized_integrals(V, dl, s)

    D = np.zeros((n_v, n_v)) if with_density else None
    parts = []
    pair_energy = np.full((n_h, n_h), np.nan)
    pair_tnorm = np.zeros((n_h, n_h))

    # core-core term: 2 t^{mn}_{ee'} tc^{mn}_{fe'}; energy weight 1/4 * 2 * 2
    for m in core:
        for n in core:
            if pair_mask is not None and not pair_mask[m, n]:
                pair_energy[m, n] = 0.0
                continue
            T, Vr = amps(m, n)
            Tc = tcheck(T)
            e = float(np.sum(Vr * Tc))
            parts.append(e)
            pair_energy[m, n] = e
            pair_tnorm[m, n] = np.linalg.norm(T)
            if with_density:
                D += 2.0 * (T @ Tc.T)

    if n_act:
        # core-active term: S(t^{mu}_{ee'} tc^{mv}_{fe'}) Gamma^u_v
        #   = sum_uv Gamma_uv (T_mu Tc_mv^T + T_um Tc_vm^T); energy weight 1/4 * 2 * Gamma_uv
        for m in core:
            T_mu, Vr_mu, T_um, Vr_um = [], [], [], []
            for u in act:
                a, b = amps(m, u)
                T_mu.append(a)
                Vr_mu.append(b)
                pair_tnorm[m, u] = np.linalg.norm(a)
                a, b = amps(u, m)
                T_um.append(a)
                Vr_um.append(b)
                pair_tnorm[u, m] = np.linalg.norm(a)
            Tc_mu = [tcheck(t) for t in T_mu]
            Tc_um = [tcheck(t) for t in T_um]
            for ui in range(n_act):
                # sum over v of Gamma_uv Tc_mv (and Tc_vm)
                mix1 = sum(G[ui, vi] * Tc_mu[vi] for vi in range(n_act))
                mix2 = sum(G[ui, vi] * Tc_um[vi] for vi in range(n_act))
                if with_density:
                    D += T_mu[ui] @ mix1.T + T_um[ui] @ mix2.T
                parts.append(0.5 * float(np.sum(Vr_mu[ui] * mix1)))
                parts.append(0.5 * float(np.sum(Vr_um[ui] * mix2)))

        # active-active term: t^{uv}_{ee'} t^{xy}_{fe'} Gamma^{uv}_{xy}
        T_aa = {}
        Vr_aa = {}
        for ui, u in enumerate(act):
            for vi, v in enumerate(act):
                T_aa[ui, vi], Vr_aa[ui, vi] = amps(u, v)
                pair_tnorm[u, v] = np.linalg.norm(T_aa[ui, vi])
        G2 = (np.einsum("ux,vy->uvxy", G, G)
              - 0.5 * np.einsum("vx,uy->uvxy", G, G))        # Gamma^{uv}_{xy}, Lambda_2 = 0
        for ui in range(n_act):
            for vi in range(n_act):
                mixT = sum(G2[ui, vi, xi, yi] * T_aa[xi, yi]
                           for xi in range(n_act) for yi in range(n_act))
                if with_density:
                    D += T_aa[ui, vi] @ mixT.T
                # energy: 1/4 Gamma_ux Gamma_vy <Vr_uv, Tc_xy>
                mixTc = sum(G[ui, xi] * G[vi, yi] * tcheck(T_aa[xi, yi])
                            for xi in range(n_act) for yi in range(n_act))
                parts.append(0.25 * float(np.sum(Vr_aa[ui, vi] * mixTc)))

    return PassResult(energy=dd_from_parts(parts), D_vv=D,
                      pair_energy=pair_energy, pair_tnorm=pair_tnorm)


def pt2_pass_inputs(inp, s: float, with_density: bool = True, pair_mask=None) -> PassResult:
    return pt2_pass(inp.eps_core, inp.eps_act, inp.eps_vir, inp.gamma_act, inp.B, s,
                    with_density=with_density, pair_mask=pair_mask)


def pair_values(inp, i: int, j: int, s: float) -> Tuple[float, float]:
    """(<Vr_ij, Tc_ij>, ||T_ij||_F) for one ordered pair, for sampled checks."""
    eps_h = inp.eps_hole
    V = pair_integrals(inp.B, i, j)
    dl = pair_denominators(eps_h, inp.eps_vir, i, j)
    T = first_order_doubles(V, dl, s)
    Vr = renormalized_integrals(V, dl, s)
    return float(np.sum(Vr * tcheck(T))), float(np.linalg.norm(T))


# ----------------------------------------------------------------------------
# Natural orbitals and truncation (Sec. 2, Eqs. 8-10)
# ----------------------------------------------------------------------------


def natural_orbitals(D: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Gamma V = n V (Eq. 8).  Returns ONs in descending order and the NOs as
    columns, each oriented so that its largest-magnitude component is positive."""
    w, v = np.linalg.eigh(D)
    order = np.argsort(-w, kind="stable")
    w, v = w[order], v[:, order]
    piv = np.argmax(np.abs(v), axis=0)
    sgn = np.sign(v[piv, np.arange(v.shape[1])])
    sgn[sgn == 0] = 1.0
    return w, v * sgn[None, :]


def cumulative_fraction(occ_desc: np.ndarray) -> np.ndarray:
    """c_k = sum_{p<=k} n_p / sum_p n_p, the p_o of Eq. 10 for k kept NOs."""
    c = np.cumsum(occ_desc)
    return c / c[-1]


def kept_count_po(occ_desc: np.ndarray, p_o: float) -> Tuple[int, Tuple[float, float]]:
    """Smallest N' whose cumulative ON fraction reaches p_o (Eq. 10).

    The comparison is c_k >= p_o * total with total the last prefix sum, so
    p_o = 1 keeps every virtual.  Margins are (p_o - c_{N'-1}, c_{N'} - p_o)
    as fractions of the total."""
    if not (0.0 < p_o <= 1.0):
        raise ValueError("p_o must lie in (0, 1]")
    c = np.cumsum(occ_desc)
    total = c[-1]
    idx = int(np.argmax(c >= p_o * total))
    n_kept = idx + 1
    below = p_o - (c[idx - 1] / total if idx >= 1 else 0.0)
    above = c[idx] / total - p_o
    return n_kept, (below, above)


def kept_count_pv(n_vir: int, p_v: float) -> int:
    """N' from a retained-virtual fraction p_v = N'/N_V (Eq. 9), rounded up."""
    if not (0.0 < p_v <= 1.0):
        raise ValueError("p_v must lie in (0, 1]")
    return int(min(n_vir, math.ceil(p_v * n_vir - 1e-9)))


def kept_count_cutoff(occ_desc: np.ndarray, n_kappa: float) -> int:
    """Number of NOs whose ON is not smaller than the cutoff n_kappa (Sec. 2)."""
    return int(np.sum(occ_desc >= n_kappa))


def expand_near_degenerate(occ_desc: np.ndarray, n_kept: int, rel_tol: float) -> int:
    """Near-degeneracy expansion (Sec. 2, after Eq. 10), anchored reading: keep
    adding NOs p beyond the cut while n_last - n_p < rel_tol * n_last, where
    n_last is the smallest ON the threshold kept.  rel_tol = 0 disables it."""
    if rel_tol <= 0.0 or n_kept >= occ_desc.shape[0]:
        return n_kept
    n_last = occ_desc[n_kept - 1]
    k = n_kept
    while k < occ_desc.shape[0] and (n_last - occ_desc[k]) < rel_tol * n_last:
        k += 1
    return k


# ----------------------------------------------------------------------------
# Recanonicalization, kept-space energy and the additive correction
# (Sec. 2: rebuild in the reduced set, recanonicalize; Eq. 11)
# ----------------------------------------------------------------------------


def recanonicalize(no_kept: np.ndarray, eps_vir: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Diagonalize the virtual Fock block in the kept NO space.

    F' = V_k^T diag(eps_v) V_k = W diag(eps~) W^T; returns (U = V_k W, eps~) with
    eps~ ascending."""
    F = no_kept.T @ (eps_vir[:, None] * no_kept)
    F = 0.5 * (F + F.T)
    et, W = np.linalg.eigh(F)
    return no_kept @ W, et


def transform_b(B: np.ndarray, U: np.ndarray) -> np.ndarray:
    """B~^Q_{ia'} = sum_a B^Q_ia U_{aa'} in the [hole, virtual, aux] layout."""
    return np.matmul(U.T[None, :, :], B)


def kept_energy(inp, no_vecs: np.ndarray, n_kept: int, s: float) -> Tuple[float, float]:
    """E_PT2 in the recanonicalized kept NO basis."""
    U, et = recanonicalize(no_vecs[:, :n_kept], inp.eps_vir)
    Bt = transform_b(inp.B, U)
    r = pt2_pass(inp.eps_core, inp.eps_act, et, inp.gamma_act, Bt, s, with_density=False)
    return r.energy


def pt2_correction(e_full: Tuple[float, float], e_kept: Tuple[float, float]) -> Tuple[float, float]:
    """Scalar part of H_PT2(MO) - H_PT2(FNO) (Eq. 11)."""
    return dd_sub(e_full, e_kept)


def full_pipeline(inp, s: float, p_o: float, degen_rel_tol: float = 0.0) -> Dict:
    r = pt2_pass_inputs(inp, s)
    occ, vecs = natural_orbitals(r.D_vv)
    n_kept, margins = kept_count_po(occ, p_o)
    n_kept = expand_near_degenerate(occ, n_kept, degen_rel_tol)
    e_kept = kept_energy(inp, vecs, n_kept, s)
    return dict(energy=r.energy, D_vv=r.D_vv, occ=occ, no_vecs=vecs, n_kept=n_kept,
                margins=margins, e_kept=e_kept, correction=pt2_correction(r.energy, e_kept),
                pair_energy=r.pair_energy, pair_tnorm=r.pair_tnorm)

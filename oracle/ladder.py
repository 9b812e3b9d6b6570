"""Density-fitted particle-particle ladder in the full or a truncated virtual space.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The cost of the high-level DSRG step is dominated by the two-body contraction
C2 = [O2, T2]_2 (Eq. 6), whose particle-particle ladder part scales as
N_C^2 N_V^4; truncating the virtuals to N_V' NOs cuts it by (N_V'/N_V)^4
(Sec. 2).  For amplitude matrices T^p (one per hole pair p, virtual x virtual)
and density-fitted virtual-virtual integrals B^Q_ac the closed-shell ladder is
    (ac|bd) = sum_Q B^Q_ac B^Q_bd
    R^p_ab  = sum_cd (ac|bd) T^p_cd
In the truncated space spanned by the kept NOs X (N_V x N_V', orthonormal
columns) the same contraction runs on B'^Q = X^T B^Q X and T'^p = X^T T^p X.
"""
from __future__ import annotations

import numpy as np


def four_index(B_vv: np.ndarray) -> np.ndarray:
    """(ac|bd) as an [a, c, b, d] array from B_vv [a, c, Q] (small sizes only)."""
    return np.einsum("acQ,bdQ->acbd", B_vv, B_vv, optimize=True)


def pp_ladder(B_vv: np.ndarray, T: np.ndarray) -> np.ndarray:
    """R [p, a, b] = sum_cd (ac|bd) T[p, c, d], through the explicit four-index integrals."""
    return np.einsum("acbd,pcd->pab", four_index(B_vv), T, optimize=True)


def transform_to_kept(B_vv: np.ndarray, T: np.ndarray, X: np.ndarray):
    """B'^Q = X^T B^Q X and T'^p = X^T T^p X for kept NOs X [n_vir, n_kept]."""
    Bk = np.einsum("ai,cj,acQ->ijQ", X, X, B_vv, optimize=True)
    Tk = np.einsum("ai,bj,pab->pij", X, X, T, optimize=True)
    return Bk, Tk


def pp_ladder_kept(B_vv: np.ndarray, T: np.ndarray, X: np.ndarray) -> np.ndarray:
    """The ladder in the space of the kept NOs (R' [p, n_kept, n_kept])."""
    Bk, Tk = transform_to_kept(B_vv, T, X)
    return pp_ladder(Bk, Tk)

"""Natural auxiliary functions for the density-fitted integrals of the pass.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's conclusions propose reducing the auxiliary dimension with natural
auxiliary functions (NAF, Kallay 2014) and expect it to speed up the DSRG-PT2
step that builds the 1-RDM.  With the three-index integrals written as the
matrix J[(i,a), P] = B^P_ia over every hole i and virtual a:
    W = J^T J                           (n_aux x n_aux, symmetric PSD)
    W = U diag(sigma) U^T               (sigma descending)
    keep the k with sigma_k > eps sigma_0   (relative threshold; eps <= 0 keeps all)
    B~^k_ia = sum_P B^P_ia U_Pk         (the compressed integrals)
Then V_ij = B_i B_j^T becomes B~_i B~_j^T; it is exact when every function is
kept (U orthogonal), and sum_ia ||B_ia||^2 - sum_ia ||B~_ia||^2 equals the sum of
the dropped sigma_k.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def naf_compress(B: np.ndarray, eps: float) -> Tuple[np.ndarray, np.ndarray, int]:
    """B [n_h, n_v, n_aux] -> (B~ [n_h, n_v, n_naf], sigma [n_aux] descending, n_naf);
    eps is relative to the largest eigenvalue sigma_0."""
    n_h, n_v, n_aux = B.shape
    J = B.reshape(n_h * n_v, n_aux)
    W = J.T @ J
    w, U = np.linalg.eigh(W)
    sigma = w[::-1].copy()
    U = U[:, ::-1]
    n_naf = n_aux if eps <= 0.0 else int(np.sum(sigma > eps * sigma[0]))
    Bt = (J @ U[:, :n_naf]).reshape(n_h, n_v, n_naf)
    return Bt, sigma, n_naf

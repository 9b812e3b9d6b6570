"""Seeded synthetic inputs for the DF-DSRG-PT2 virtual-density pass.

This module is shared by the FP64 oracle, the tests and the benchmark.  It draws
random numbers and lays them out; it holds none of the method's arithmetic (no
integrals, amplitudes, energies or densities are formed here).

Inputs of the pass (paper Sec. 2 and App. A):
  * semicanonical orbital energies of the correlated core holes, of the active
    holes and of the virtuals (the diagonal Fock blocks of Eq. A5),
  * the spin-summed active one-body density Gamma_act (Eq. A1), symmetric,
    eigenvalues in [0, 2],
  * density-fitted three-index integrals B^Q_ia for holes i and virtuals a
    (the paper uses DF integrals with one common auxiliary basis, Sec. 3).

The molecules of the paper are not available, so every input is drawn from the
distributions below, shaped like the paper's workloads (Sec. 3: Ni(CO)4 with
N_V = 539 virtuals; FeCl(Cor) with more than 1000 basis functions).

Recipe (random stream ``numpy.random.default_rng(seed)``, PCG64), draws in
this order:
  1. core (or closed-shell occupied) energies  U[-1.5, -0.3] Eh, sorted ascending
  2. virtual energies                          U[ 0.1,  5.0] Eh, sorted ascending
  3. (active space only) active energies       U[-0.3,  0.0] Eh, sorted ascending
     then x ~ U[0, 2]^(n_act/2) and a standard-normal n_act x n_act matrix G;
     Gamma_act = Q diag(x, 2 - x) Q^T with Q from the QR factorization of G,
     columns signed so that R has a positive diagonal (Haar-distributed Q);
     trace(Gamma_act) = n_act exactly.
  4. Z ~ N(0, 1) with C-order shape (n_aux, n_h, n_v)
  5. (low-rank variant only) P ~ N(0,1)^(n_aux x 64), R ~ N(0,1)^(64 x n_h*n_v)
  6. (localized variant only) hole positions x_i ~ U[0, 40], aux positions
     y_Q ~ U[0, 40]
  7. (redundant-auxiliary variant only, rank r) C ~ N(0,1)^(n_aux x r),
     Y ~ N(0,1)^(r x n_h*n_v); Z is then scaled by the noise level nu
  B^Q_ia = d_a * (Z^Q_ia [+ (P R)^Q_ia / 8]) [* exp(-|x_i - y_Q| / xi)],
  with the virtual decay d_a = 0.3 / (1 + eps_a) * 0.2; in the redundant-auxiliary
  variant B^Q_ia = d_a * ((C Y)^Q_ia / sqrt(r) + nu Z^Q_ia): n_aux functions that
  span only an r-dimensional space up to noise, the situation of a large
  automatically generated auxiliary set that natural auxiliary functions compress.

Active-particle integrals (``active_particles=True``, drawn after everything
above from the same stream): Z' ~ N(0,1) with C-order shape (n_aux, n_h, n_act),
B_act^Q_ix = d_x Z'^Q_ix with the decay d_x of the active orbital energies, then
the active-hole / active-particle block symmetrized, B^Q_{n_c+u, x} and
B^Q_{n_c+x, u} both replaced by their sum over sqrt(2) (B^Q_ux = B^Q_xu, as
density-fitted integrals are).

Two-body density cumulant of the active orbitals (``active_cumulant``, a
separate stream ``default_rng(seed)``): G ~ N(0,1) with shape (n_act,)*4, made
symmetric under the simultaneous swap of both index pairs and under the exchange
of the pairs, lambda = c (G + G^(vu yx)) / 2 then (lambda + lambda^(xy uv)) / 2,
with c = 0.1 (the size of the cumulants of a correlated few-electron reference;
no other structure is imposed, the terms that consume it being linear in it).

Particle-particle ladder inputs (``ladder_inputs``, a separate stream
``default_rng(seed)``): virtual energies U[0.1, 5.0] sorted; Z ~ N(0,1) with
C-order shape (n_aux, n_v, n_v); W ~ N(0,1) with shape (n_amp, n_v, n_v);
  B^Q_ac = sqrt(d_a d_c) (Z^Q_ac + Z^Q_ca) / sqrt(2)   (symmetric in a, c, as
           density-fitted virtual-virtual integrals are)
  T^p_cd = 0.05 W^p_cd / (1 + eps_c + eps_d)          (amplitude-sized matrices)
with the same decay d_a as above.

Holes are ordered core first, then active.  B is returned in the layout the
library consumes, ``B[i, a, Q]`` (hole, virtual, auxiliary; auxiliary fastest),
FP64, C-contiguous.  It is filled chunk by chunk over Q from the same random
stream, so the values do not depend on the chunk size.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = ["Inputs", "generate", "CONFIGS", "config_inputs", "input_recipe", "mlp_init", "active_cumulant"]


@dataclasses.dataclass
class Inputs:
    eps_core: np.ndarray          # [n_core]
    eps_act: np.ndarray           # [n_act]
    eps_vir: np.ndarray           # [n_vir], ascending
    gamma_act: np.ndarray         # [n_act, n_act], symmetric (empty if n_act == 0)
    B: np.ndarray                 # [n_h, n_vir, n_aux]
    seed: int = 0
    label: str = ""
    B_act: Optional[np.ndarray] = None  # [n_h, n_act, n_aux] hole / active-particle integrals, or None

    @property
    def n_core(self) -> int:
        return int(self.eps_core.shape[0])

    @property
    def n_act(self) -> int:
        return int(self.eps_act.shape[0])

    @property
    def n_h(self) -> int:
        return self.n_core + self.n_act

    @property
    def n_vir(self) -> int:
        return int(self.eps_vir.shape[0])

    @property
    def n_aux(self) -> int:
        return int(self.B.shape[2])

    @property
    def eps_hole(self) -> np.ndarray:
        return np.concatenate([self.eps_core, self.eps_act])

    def replace(self, **kw) -> "Inputs":
        return dataclasses.replace(self, **kw)


def _haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def generate(n_core: int, n_act: int, n_vir: int, n_aux: int, seed: int = 0, *,
             low_rank: int = 0, localized_xi: Optional[float] = None,
             aux_rank: int = 0, aux_noise: float = 0.0, active_particles: bool = False,
             q_chunk: int = 256, label: str = "") -> Inputs:
    """Draw one input set following the recipe in the module docstring."""
    if n_act % 2:
        raise ValueError("n_act must be even (eigenvalues come in pairs x, 2-x)")
    rng = np.random.default_rng(seed)
    eps_core = np.sort(rng.uniform(-1.5, -0.3, n_core))
    eps_vir = np.sort(rng.uniform(0.1, 5.0, n_vir))
    if n_act:
        eps_act = np.sort(rng.uniform(-0.3, 0.0, n_act))
        x = rng.uniform(0.0, 2.0, n_act // 2)
        q = _haar_orthogonal(rng, n_act)
        lam = np.concatenate([x, 2.0 - x])
        gamma = (q * lam[None, :]) @ q.T
        gamma = 0.5 * (gamma + gamma.T)
    else:
        eps_act = np.zeros(0)
        gamma = np.zeros((0, 0))
    n_h = n_core + n_act
    d = 0.3 / (1.0 + eps_vir) * 0.2                     # virtual decay d_a
    B = np.empty((n_h, n_vir, n_aux), dtype=np.float64)
    for q0 in range(0, n_aux, q_chunk):
        q1 = min(n_aux, q0 + q_chunk)
        z = rng.standard_normal((q1 - q0, n_h, n_vir))
        B[:, :, q0:q1] = z.transpose(1, 2, 0)
    if low_rank:
        p = rng.standard_normal((n_aux, low_rank))
        r = rng.standard_normal((low_rank, n_h * n_vir))
        scale = 1.0 / np.sqrt(low_rank)
        for q0 in range(0, n_aux, q_chunk):
            q1 = min(n_aux, q0 + q_chunk)
            add = (p[q0:q1] @ r).reshape(q1 - q0, n_h, n_vir) * scale
            B[:, :, q0:q1] += add.transpose(1, 2, 0)
    if aux_rank:
        B *= aux_noise
        c = rng.standard_normal((n_aux, aux_rank))
        y = rng.standard_normal((aux_rank, n_h * n_vir))
        scale = 1.0 / np.sqrt(aux_rank)
        for q0 in range(0, n_aux, q_chunk):
            q1 = min(n_aux, q0 + q_chunk)
            add = (c[q0:q1] @ y).reshape(q1 - q0, n_h, n_vir) * scale
            B[:, :, q0:q1] += add.transpose(1, 2, 0)
    B *= d[None, :, None]
    if localized_xi is not None:
        xh = rng.uniform(0.0, 40.0, n_h)
        yq = rng.uniform(0.0, 40.0, n_aux)
        B *= np.exp(-np.abs(xh[:, None] - yq[None, :]) / localized_xi)[:, None, :]
    B_act = None
    if active_particles and n_act:
        z = rng.standard_normal((n_aux, n_h, n_act))
        dx = 0.3 / (1.0 + eps_act) * 0.2
        B_act = np.ascontiguousarray(z.transpose(1, 2, 0) * dx[None, :, None])
        blk = B_act[n_core:].copy()
        B_act[n_core:] = (blk + blk.transpose(1, 0, 2)) / np.sqrt(2.0)
    return Inputs(eps_core=eps_core, eps_act=eps_act, eps_vir=eps_vir,
                  gamma_act=gamma, B=B, seed=seed, label=label, B_act=B_act)


# Workload presets.  Sizes are (n_core, n_act, n_vir, n_aux).
CONFIGS = {
    # closed shell, small enough for the oracle in well under a second
    "c1": dict(sizes=(10, 0, 60, 200), s=(0.5,), p_o=(0.985,), precision="fp64",
               gen=dict()),
    # active space (trace-8 Gamma_act) and a rank-64 shared component in B
    "c2": dict(sizes=(40, 8, 400, 1600), s=(0.5,), p_o=(0.98, 0.985, 0.99),
               precision="fp64", gen=dict(low_rank=64)),
    # ~1300 basis functions, closed shell, split-BF16 GEMMs
    "c3": dict(sizes=(80, 0, 1200, 4000), s=(0.5, 1.0), p_o=(0.985,),
               precision="bf16", gen=dict()),
    # learned pair screening: train at c1 sizes over seeds 1..200, apply at c3 sizes
    "c4": dict(sizes=(80, 0, 1200, 4000), s=(0.5,), p_o=(0.985,), precision="bf16",
               gen=dict(), train_sizes=(10, 0, 60, 200), train_seeds=(1, 200)),
    # largest one-GPU instance, trace-12 Gamma_act
    "c5": dict(sizes=(120, 12, 2000, 6000), s=(0.5,), p_o=(0.985,), precision="fp8",
               gen=dict()),
}


def config_inputs(name: str, seed: int = 0, **over) -> Inputs:
    cfg = CONFIGS[name]
    n_core, n_act, n_vir, n_aux = cfg["sizes"]
    kw = dict(cfg["gen"])
    kw.update(over)
    return generate(n_core, n_act, n_vir, n_aux, seed, label=name, **kw)


def input_recipe() -> str:
    return __doc__


def mlp_init(seed: int = 0, hidden: int = 64, n_in: int = 5) -> np.ndarray:
    """Seeded initial parameters of the pair-screen network, packed as
    [W1 (hidden x n_in), b1, W2 (hidden x hidden), b2, w3 (hidden), b3]:
    weights ~ N(0, 1/fan_in), biases 0."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((hidden, n_in)) / np.sqrt(n_in)
    W2 = rng.standard_normal((hidden, hidden)) / np.sqrt(hidden)
    w3 = rng.standard_normal(hidden) / np.sqrt(hidden)
    return np.concatenate([W1.ravel(), np.zeros(hidden), W2.ravel(), np.zeros(hidden), w3, [0.0]])


def active_cumulant(n_act: int, seed: int = 0, scale: float = 0.1) -> np.ndarray:
    """lam[u, v, x, y] (= lambda_uv^xy) following the recipe in the module docstring."""
    g = np.random.default_rng(seed).standard_normal((n_act,) * 4)
    lam = 0.5 * scale * (g + g.transpose(1, 0, 3, 2))
    return np.ascontiguousarray(0.5 * (lam + lam.transpose(2, 3, 0, 1)))


@dataclasses.dataclass
class LadderInputs:
    eps_vir: np.ndarray      # [n_v]
    B_vv: np.ndarray         # [n_v, n_v, n_aux], symmetric in the two virtual indices
    T: np.ndarray            # [n_amp, n_v, n_v]
    seed: int = 0


def ladder_inputs(n_vir: int, n_aux: int, n_amp: int, seed: int = 0) -> LadderInputs:
    """Draw the particle-particle ladder inputs following the recipe in the module docstring."""
    rng = np.random.default_rng(seed)
    eps_vir = np.sort(rng.uniform(0.1, 5.0, n_vir))
    d = 0.3 / (1.0 + eps_vir) * 0.2
    z = rng.standard_normal((n_aux, n_vir, n_vir))
    s = (z + z.transpose(0, 2, 1)) / np.sqrt(2.0)
    B = np.ascontiguousarray((s * np.sqrt(np.outer(d, d))[None, :, :]).transpose(1, 2, 0))
    w = rng.standard_normal((n_amp, n_vir, n_vir))
    T = 0.05 * w / (1.0 + eps_vir[None, :, None] + eps_vir[None, None, :])
    return LadderInputs(eps_vir=eps_vir, B_vv=B, T=np.ascontiguousarray(T), seed=seed)

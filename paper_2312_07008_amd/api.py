"""Python binding of libdfpt2.so: argument marshalling only.

Every entry point mirrors the C function of the same name in include/dfpt2.h.
Tensors must already live on the GPU; torch provides device memory and the
current stream and nothing else.  Outputs not passed in are allocated with
torch.empty on the device of the inputs.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import Opts, check

__all__ = ["make_opts", "add_cumulant_singles_density", "workspace_size", "build_vv_density", "build_vv_density_noalloc", "fno_truncate_workspace_size",
           "fno_truncate", "fno_truncate_rule", "naf_compress", "eigh_sym", "pt2_correction_workspace_size", "pt2_energy_correction",
           "upload_inputs", "profile_enable", "profile_read", "pp_ladder", "pp_ladder_workspace_size",
           "add_active_particle_density", "pairscreen_num_params", "pairscreen_features",
           "pairscreen_mlp_forward", "pairscreen_mlp_backward", "pairscreen_adam_step", "pairscreen_train",
           "pairscreen_targets", "pairscreen_build_mask"]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype, numel: int):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def make_opts(n_core: int, n_act: int, n_vir: int, n_aux: int, s: float, precision: int = _lib.FP64,
              slices_gemm1: int = 0, slices_gemm2: int = 0, density_convention: int = 0,
              pair_batch: int = 0) -> Opts:
    return Opts(n_core, n_act, n_vir, n_aux, float(s), precision, slices_gemm1, slices_gemm2,
                density_convention, pair_batch)


def workspace_size(opts: Opts) -> int:
    lib = _lib.load()
    n = ctypes.c_size_t(0)
    check(lib.dfpt2_workspace_size(ctypes.byref(opts), ctypes.byref(n)))
    return int(n.value)


def _workspace(nbytes: int, device, workspace: Optional[torch.Tensor]):
    if workspace is not None:
        if workspace.device.type != "cuda" or workspace.dtype != torch.uint8:
            raise TypeError("workspace must be a uint8 GPU tensor")
        return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def build_vv_density(opts: Opts, eps_hole: torch.Tensor, eps_vir: torch.Tensor,
                     gamma_act: Optional[torch.Tensor], B: torch.Tensor,
                     pair_mask: Optional[torch.Tensor] = None, *, D_vv=None, e_pt2=None,
                     pair_energy=None, pair_tnorm=None, want_pair_energy: bool = False,
                     want_pair_tnorm: bool = False, workspace=None, stream=None) -> dict:
    lib = _lib.load()
    n_h = opts.n_core + opts.n_act
    n_v, n_aux = opts.n_vir, opts.n_aux
    _need(eps_hole, "eps_hole", torch.float64, n_h)
    _need(eps_vir, "eps_vir", torch.float64, n_v)
    _need(B, "B", torch.float64, n_h * n_v * n_aux)
    if opts.n_act:
        _need(gamma_act, "gamma_act", torch.float64, opts.n_act * opts.n_act)
    else:
        gamma_act = None
    if pair_mask is not None:
        _need(pair_mask, "pair_mask", torch.uint8, n_h * n_h)
    dev = B.device
    if D_vv is None:
        D_vv = torch.empty((n_v, n_v), dtype=torch.float64, device=dev)
    if e_pt2 is None:
        e_pt2 = torch.empty(2, dtype=torch.float64, device=dev)
    if pair_energy is None and want_pair_energy:
        pair_energy = torch.empty((n_h, n_h), dtype=torch.float64, device=dev)
    if pair_tnorm is None and want_pair_tnorm:
        pair_tnorm = torch.empty((n_h, n_h), dtype=torch.float32, device=dev)
    _need(D_vv, "D_vv", torch.float64, n_v * n_v)
    _need(e_pt2, "e_pt2", torch.float64, 2)
    if pair_energy is not None:
        _need(pair_energy, "pair_energy", torch.float64, n_h * n_h)
    if pair_tnorm is not None:
        _need(pair_tnorm, "pair_tnorm", torch.float32, n_h * n_h)
    nbytes = workspace_size(opts)
    ws = _workspace(nbytes, dev, workspace)
    check(lib.dfpt2_build_vv_density(ctypes.byref(opts), _ptr(eps_hole), _ptr(eps_vir), _ptr(gamma_act),
                                     _ptr(B), _ptr(pair_mask), _ptr(D_vv), _ptr(e_pt2), _ptr(pair_energy),
                                     _ptr(pair_tnorm), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                     _stream(stream)))
    return dict(D_vv=D_vv, e_pt2=e_pt2, pair_energy=pair_energy, pair_tnorm=pair_tnorm)


def build_vv_density_noalloc(opts: Opts, eps_hole: torch.Tensor, eps_vir: torch.Tensor,
                             gamma_act: Optional[torch.Tensor], B: torch.Tensor,
                             pair_mask: Optional[torch.Tensor] = None, *, D_vv: torch.Tensor,
                             e_pt2: torch.Tensor, pair_energy=None, pair_tnorm=None, stream=None) -> dict:
    """dfpt2_build_vv_density_noalloc: the pass in the library's static scratch.
    Every output is caller-provided (nothing is allocated here either)."""
    lib = _lib.load()
    n_h = opts.n_core + opts.n_act
    n_v, n_aux = opts.n_vir, opts.n_aux
    _need(eps_hole, "eps_hole", torch.float64, n_h)
    _need(eps_vir, "eps_vir", torch.float64, n_v)
    _need(B, "B", torch.float64, n_h * n_v * n_aux)
    if opts.n_act:
        _need(gamma_act, "gamma_act", torch.float64, opts.n_act * opts.n_act)
    else:
        gamma_act = None
    if pair_mask is not None:
        _need(pair_mask, "pair_mask", torch.uint8, n_h * n_h)
    _need(D_vv, "D_vv", torch.float64, n_v * n_v)
    _need(e_pt2, "e_pt2", torch.float64, 2)
    if pair_energy is not None:
        _need(pair_energy, "pair_energy", torch.float64, n_h * n_h)
    if pair_tnorm is not None:
        _need(pair_tnorm, "pair_tnorm", torch.float32, n_h * n_h)
    check(lib.dfpt2_build_vv_density_noalloc(ctypes.byref(opts), _ptr(eps_hole), _ptr(eps_vir), _ptr(gamma_act),
                                             _ptr(B), _ptr(pair_mask), _ptr(D_vv), _ptr(e_pt2), _ptr(pair_energy),
                                             _ptr(pair_tnorm), _stream(stream)))
    return dict(D_vv=D_vv, e_pt2=e_pt2, pair_energy=pair_energy, pair_tnorm=pair_tnorm)


def fno_truncate_workspace_size(n_vir: int) -> int:
    lib = _lib.load()
    n = ctypes.c_size_t(0)
    check(lib.fno_truncate_workspace_size(n_vir, ctypes.byref(n)))
    return int(n.value)


def fno_truncate(D_vv: torch.Tensor, p_o: float, degen_rel_tol: float = 0.0, *, occ=None, no_vecs=None,
                 workspace=None, stream=None) -> dict:
    lib = _lib.load()
    n_v = D_vv.shape[0]
    _need(D_vv, "D_vv", torch.float64, n_v * n_v)
    dev = D_vv.device
    if occ is None:
        occ = torch.empty(n_v, dtype=torch.float64, device=dev)
    if no_vecs is None:
        no_vecs = torch.empty((n_v, n_v), dtype=torch.float64, device=dev)
    _need(occ, "occ", torch.float64, n_v)
    _need(no_vecs, "no_vecs", torch.float64, n_v * n_v)
    ws = _workspace(fno_truncate_workspace_size(n_v), dev, workspace)
    n_kept = ctypes.c_int64(0)
    margins = (ctypes.c_double * 2)()
    check(lib.fno_truncate(_ptr(D_vv), n_v, float(p_o), float(degen_rel_tol), _ptr(occ), _ptr(no_vecs),
                           ctypes.byref(n_kept), margins, _ptr(ws), ctypes.c_size_t(ws.numel()),
                           _stream(stream)))
    return dict(occ=occ, no_vecs=no_vecs, n_kept=int(n_kept.value), margins=(margins[0], margins[1]))


def fno_truncate_rule(D_vv: torch.Tensor, rule: int, param: float, degen_rel_tol: float = 0.0, *, occ=None,
                      no_vecs=None, workspace=None, stream=None) -> dict:
    """fno_truncate with an explicit rule (TRUNC_CUMULATIVE p_o, TRUNC_FRACTION p_v,
    TRUNC_CUTOFF n_kappa, TRUNC_FIXED N')."""
    lib = _lib.load()
    n_v = D_vv.shape[0]
    _need(D_vv, "D_vv", torch.float64, n_v * n_v)
    dev = D_vv.device
    if occ is None:
        occ = torch.empty(n_v, dtype=torch.float64, device=dev)
    if no_vecs is None:
        no_vecs = torch.empty((n_v, n_v), dtype=torch.float64, device=dev)
    _need(occ, "occ", torch.float64, n_v)
    _need(no_vecs, "no_vecs", torch.float64, n_v * n_v)
    ws = _workspace(fno_truncate_workspace_size(n_v), dev, workspace)
    n_kept = ctypes.c_int64(0)
    margins = (ctypes.c_double * 2)()
    check(lib.fno_truncate_rule(_ptr(D_vv), n_v, int(rule), float(param), float(degen_rel_tol), _ptr(occ),
                                _ptr(no_vecs), ctypes.byref(n_kept), margins, _ptr(ws), ctypes.c_size_t(ws.numel()),
                                _stream(stream)))
    return dict(occ=occ, no_vecs=no_vecs, n_kept=int(n_kept.value), margins=(margins[0], margins[1]))


def naf_compress(opts, B: torch.Tensor, eps: float, *, workspace=None, stream=None) -> dict:
    """Natural auxiliary functions: returns B_naf [n_h, n_vir, n_naf], sigma [n_aux]
    (descending) and n_naf."""
    lib = _lib.load()
    n_h, n_v, n_aux = opts.n_core + opts.n_act, opts.n_vir, opts.n_aux
    _need(B, "B", torch.float64, n_h * n_v * n_aux)
    dev = B.device
    out = torch.empty(n_h * n_v * n_aux, dtype=torch.float64, device=dev)
    sigma = torch.empty(n_aux, dtype=torch.float64, device=dev)
    n = ctypes.c_size_t(0)
    check(lib.naf_compress_workspace_size(ctypes.byref(opts), ctypes.byref(n)))
    ws = _workspace(int(n.value), dev, workspace)
    k = ctypes.c_int64(0)
    check(lib.naf_compress(ctypes.byref(opts), _ptr(B), float(eps), _ptr(out), _ptr(sigma), ctypes.byref(k),
                           _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(stream)))
    k = int(k.value)
    return dict(B_naf=out[: n_h * n_v * k].view(n_h, n_v, k), sigma=sigma, n_naf=k)


def add_active_particle_density(opts: Opts, eps_hole, eps_vir, gamma_act, B, B_act, D_vv, *, workspace=None,
                                stream=None) -> torch.Tensor:
    """D_vv += the Eq. A9 terms with an active particle index (zero cumulants); returns D_vv."""
    lib = _lib.load()
    n_h, n_v, n_a, n_aux = opts.n_core + opts.n_act, opts.n_vir, opts.n_act, opts.n_aux
    _need(eps_hole, "eps_hole", torch.float64, n_h)
    _need(eps_vir, "eps_vir", torch.float64, n_v)
    _need(gamma_act, "gamma_act", torch.float64, n_a * n_a)
    _need(B, "B", torch.float64, n_h * n_v * n_aux)
    _need(B_act, "B_act", torch.float64, n_h * n_a * n_aux)
    _need(D_vv, "D_vv", torch.float64, n_v * n_v)
    n = ctypes.c_size_t(0)
    check(lib.dfpt2_active_particle_workspace_size(ctypes.byref(opts), ctypes.byref(n)))
    ws = _workspace(int(n.value), D_vv.device, workspace)
    check(lib.dfpt2_add_active_particle_density(ctypes.byref(opts), _ptr(eps_hole), _ptr(eps_vir), _ptr(gamma_act),
                                                _ptr(B), _ptr(B_act), _ptr(D_vv), _ptr(ws),
                                                ctypes.c_size_t(ws.numel()), _stream(stream)))
    return D_vv


def add_cumulant_singles_density(opts: Opts, eps_hole, eps_vir, gamma_act, lambda_act, B, B_act, D_vv, *,
                                 t1=None, workspace=None, stream=None) -> torch.Tensor:
    """D_vv += the Eq. A9 terms with the singles (Eq. A6) and, if lambda_act is given,
    with the two-body cumulant; t1 [n_h, n_vir] (optional) receives the singles."""
    lib = _lib.load()
    n_h, n_v, n_a, n_aux = opts.n_core + opts.n_act, opts.n_vir, opts.n_act, opts.n_aux
    _need(eps_hole, "eps_hole", torch.float64, n_h)
    _need(eps_vir, "eps_vir", torch.float64, n_v)
    _need(gamma_act, "gamma_act", torch.float64, n_a * n_a)
    if lambda_act is not None:
        _need(lambda_act, "lambda_act", torch.float64, n_a ** 4)
    _need(B, "B", torch.float64, n_h * n_v * n_aux)
    _need(B_act, "B_act", torch.float64, n_h * n_a * n_aux)
    _need(D_vv, "D_vv", torch.float64, n_v * n_v)
    if t1 is not None:
        _need(t1, "t1", torch.float64, n_h * n_v)
    n = ctypes.c_size_t(0)
    check(lib.dfpt2_cumulant_singles_workspace_size(ctypes.byref(opts), int(lambda_act is not None), ctypes.byref(n)))
    ws = _workspace(int(n.value), D_vv.device, workspace)
    check(lib.dfpt2_add_cumulant_singles_density(ctypes.byref(opts), _ptr(eps_hole), _ptr(eps_vir), _ptr(gamma_act),
                                                 _ptr(lambda_act), _ptr(B), _ptr(B_act), _ptr(D_vv), _ptr(t1),
                                                 _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(stream)))
    return D_vv


def pp_ladder_workspace_size(n_vir: int, n_aux: int, n_amp: int, n_kept: int = 0) -> int:
    lib = _lib.load()
    n = ctypes.c_size_t(0)
    check(lib.pp_ladder_workspace_size(n_vir, n_aux, n_amp, n_kept, ctypes.byref(n)))
    return int(n.value)


def pp_ladder(B_vv: torch.Tensor, T: torch.Tensor, X: Optional[torch.Tensor] = None, n_kept: int = 0, *,
              R: Optional[torch.Tensor] = None, workspace=None, stream=None) -> torch.Tensor:
    """Particle-particle ladder R^p_ab = sum_cd (ac|bd) T^p_cd; with X [n_vir, ldx] (its first
    n_kept columns are the kept NOs, e.g. fno_truncate's no_vecs) in the truncated space.
    Returns R [n_amp, m, m]."""
    lib = _lib.load()
    n_v, n_aux = B_vv.shape[0], B_vv.shape[2]
    n_amp = T.shape[0]
    _need(B_vv, "B_vv", torch.float64, n_v * n_v * n_aux)
    _need(T, "T", torch.float64, n_amp * n_v * n_v)
    if X is not None:
        if n_kept < 1:
            raise ValueError("n_kept must be given with X")
        if X.dim() != 2 or X.shape[0] != n_v or X.shape[1] < n_kept:
            raise ValueError("X must be [n_vir, ldx] with ldx >= n_kept")
        _need(X, "X", torch.float64, X.numel())
        ldx, m = X.shape[1], n_kept
    else:
        n_kept, m, ldx = 0, n_v, 0
    if R is None:
        R = torch.empty((n_amp, m, m), dtype=torch.float64, device=B_vv.device)
    _need(R, "R", torch.float64, n_amp * m * m)
    ws = _workspace(pp_ladder_workspace_size(n_v, n_aux, n_amp, n_kept), B_vv.device, workspace)
    check(lib.pp_ladder(n_v, n_aux, n_amp, _ptr(B_vv), _ptr(T), _ptr(X), ldx, n_kept, _ptr(R), _ptr(ws),
                        ctypes.c_size_t(ws.numel()), _stream(stream)))
    return R


def eigh_sym(A: torch.Tensor, *, workspace=None, stream=None):
    lib = _lib.load()
    n = A.shape[0]
    _need(A, "A", torch.float64, n * n)
    w = torch.empty(n, dtype=torch.float64, device=A.device)
    Z = torch.empty((n, n), dtype=torch.float64, device=A.device)
    ws = _workspace(fno_truncate_workspace_size(n), A.device, workspace)
    check(lib.dfpt2_eigh_sym(_ptr(A), n, _ptr(w), _ptr(Z), _ptr(ws), ctypes.c_size_t(ws.numel()),
                             _stream(stream)))
    return w, Z


def pt2_correction_workspace_size(opts: Opts, n_kept: int) -> int:
    lib = _lib.load()
    n = ctypes.c_size_t(0)
    check(lib.pt2_correction_workspace_size(ctypes.byref(opts), n_kept, ctypes.byref(n)))
    return int(n.value)


def pt2_energy_correction(opts: Opts, eps_hole, eps_vir, gamma_act, B, no_vecs, n_kept: int, e_full,
                          *, workspace=None, stream=None) -> dict:
    lib = _lib.load()
    n_h = opts.n_core + opts.n_act
    n_v, n_aux = opts.n_vir, opts.n_aux
    _need(eps_hole, "eps_hole", torch.float64, n_h)
    _need(eps_vir, "eps_vir", torch.float64, n_v)
    _need(B, "B", torch.float64, n_h * n_v * n_aux)
    _need(no_vecs, "no_vecs", torch.float64, n_v * n_v)
    _need(e_full, "e_full", torch.float64, 2)
    if opts.n_act:
        _need(gamma_act, "gamma_act", torch.float64, opts.n_act * opts.n_act)
    else:
        gamma_act = None
    dev = B.device
    e_kept = torch.empty(2, dtype=torch.float64, device=dev)
    corr = torch.empty(2, dtype=torch.float64, device=dev)
    ws = _workspace(pt2_correction_workspace_size(opts, n_kept), dev, workspace)
    check(lib.pt2_energy_correction(ctypes.byref(opts), _ptr(eps_hole), _ptr(eps_vir), _ptr(gamma_act), _ptr(B),
                                    _ptr(no_vecs), int(n_kept), _ptr(e_full), _ptr(e_kept), _ptr(corr), _ptr(ws),
                                    ctypes.c_size_t(ws.numel()), _stream(stream)))
    return dict(e_kept=e_kept, correction=corr)


def upload_inputs(inp, device="cuda") -> dict:
    """Copy a synthetic input set (numpy, layout [hole][virtual][aux]) to the GPU."""
    def t(x):
        return torch.from_numpy(x).to(device=device, dtype=torch.float64).contiguous()
    out = dict(eps_hole=t(inp.eps_hole), eps_vir=t(inp.eps_vir), B=t(inp.B))
    out["gamma_act"] = t(inp.gamma_act.reshape(-1)) if inp.n_act else None
    if getattr(inp, "B_act", None) is not None:
        out["B_act"] = t(inp.B_act)
    return out


def profile_enable(on: bool = True) -> None:
    """Turn the library's stage timers on (resetting them) or off."""
    check(_lib.load().dfpt2_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{stage: (milliseconds, timed launches)} accumulated since profile_enable."""
    n = len(_lib.STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    check(_lib.load().dfpt2_profile_read(ms, cnt))
    return {name: (ms[i], int(cnt[i])) for i, name in enumerate(_lib.STAGES)}


# ----------------------------------------------------------------- pair screening

def pairscreen_num_params() -> int:
    return int(_lib.load().pairscreen_num_params())


def pairscreen_features(opts: Opts, eps_hole, eps_vir, B, *, workspace=None, stream=None):
    lib = _lib.load()
    n_h = opts.n_core + opts.n_act
    n_up = opts.n_core * (opts.n_core + 1) // 2
    _need(eps_hole, "eps_hole", torch.float64, n_h)
    _need(eps_vir, "eps_vir", torch.float64, opts.n_vir)
    _need(B, "B", torch.float64, n_h * opts.n_vir * opts.n_aux)
    dev = B.device
    feats = torch.empty((max(n_up, 1), 5), dtype=torch.float32, device=dev)
    log_scale = torch.empty((max(n_up, 1), 2), dtype=torch.float64, device=dev)
    n = ctypes.c_size_t(0)
    check(lib.pairscreen_workspace_size(ctypes.byref(opts), ctypes.byref(n)))
    ws = _workspace(int(n.value), dev, workspace)
    check(lib.pairscreen_features(ctypes.byref(opts), _ptr(eps_hole), _ptr(eps_vir), _ptr(B), _ptr(feats),
                                  _ptr(log_scale), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(stream)))
    return feats[:n_up], log_scale[:n_up]


def pairscreen_mlp_forward(W, feats, *, want_cache=False, stream=None):
    lib = _lib.load()
    n = feats.shape[0]
    _need(W, "W", torch.float32, pairscreen_num_params())
    _need(feats, "feats", torch.float32, n * 5)
    pred = torch.empty(n, dtype=torch.float32, device=feats.device)
    cache = torch.empty((n, 128), dtype=torch.float32, device=feats.device) if want_cache else None
    check(lib.pairscreen_mlp_forward(_ptr(W), _ptr(feats), n, _ptr(pred), _ptr(cache), _stream(stream)))
    return pred, cache


def pairscreen_mlp_backward(W, feats, cache, dpred, *, stream=None):
    lib = _lib.load()
    n = feats.shape[0]
    _need(W, "W", torch.float32, pairscreen_num_params())
    _need(feats, "feats", torch.float32, n * 5)
    _need(cache, "cache", torch.float32, n * 128)
    _need(dpred, "dpred", torch.float32, n)
    dW = torch.empty_like(W)
    nb = ctypes.c_size_t(0)
    check(lib.pairscreen_backward_workspace_size(n, ctypes.byref(nb)))
    ws = _workspace(int(nb.value), feats.device, None)
    check(lib.pairscreen_mlp_backward(_ptr(W), _ptr(feats), _ptr(cache), _ptr(dpred), n, _ptr(dW), _ptr(ws),
                                      ctypes.c_size_t(ws.numel()), _stream(stream)))
    return dW


def pairscreen_adam_step(W, dW, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8, *, stream=None):
    lib = _lib.load()
    for t, nm in ((W, "W"), (dW, "dW"), (m, "m"), (v, "v")):
        _need(t, nm, torch.float32, W.numel())
    check(lib.pairscreen_adam_step(_ptr(W), _ptr(dW), _ptr(m), _ptr(v), W.numel(), lr, b1, b2, eps, step,
                                   _stream(stream)))


def pairscreen_train(W, m, v, feats, y, steps: int, lr: float, step0: int = 0, *, stream=None):
    """Full-batch training on the GPU; returns the per-step losses (device tensor)."""
    lib = _lib.load()
    n = feats.shape[0]
    _need(feats, "feats", torch.float32, n * 5)
    _need(y, "y", torch.float32, n)
    for t, nm in ((W, "W"), (m, "m"), (v, "v")):
        _need(t, nm, torch.float32, pairscreen_num_params())
    losses = torch.empty(steps, dtype=torch.float32, device=feats.device)
    nb = ctypes.c_size_t(0)
    check(lib.pairscreen_train_workspace_size(n, ctypes.byref(nb)))
    ws = _workspace(int(nb.value), feats.device, None)
    check(lib.pairscreen_train(_ptr(W), _ptr(m), _ptr(v), _ptr(feats), _ptr(y), n, steps, step0, lr, _ptr(losses),
                               _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(stream)))
    return losses


def pairscreen_targets(pair_tnorm, log_scale, n_core: int, n_h: int, *, stream=None):
    lib = _lib.load()
    n_up = n_core * (n_core + 1) // 2
    _need(pair_tnorm, "pair_tnorm", torch.float32, n_h * n_h)
    _need(log_scale, "log_scale", torch.float64, 2 * n_up)
    y = torch.empty(max(n_up, 1), dtype=torch.float32, device=pair_tnorm.device)
    check(lib.pairscreen_targets(_ptr(pair_tnorm), _ptr(log_scale), n_core, n_h, _ptr(y), _stream(stream)))
    return y[:n_up]


def pairscreen_build_mask(pred, log_scale, n_core: int, n_h: int, threshold: float, margin: float = 0.0,
                          mode: int = 0, *, stream=None):
    """Returns (mask [n_h, n_h] uint8 on the device, number of dropped unordered pairs)."""
    lib = _lib.load()
    n_up = n_core * (n_core + 1) // 2
    _need(log_scale, "log_scale", torch.float64, 2 * n_up)
    if mode == 0:
        _need(pred, "pred", torch.float32, n_up)
    mask = torch.empty((n_h, n_h), dtype=torch.uint8, device=log_scale.device)
    ws = torch.empty(256, dtype=torch.uint8, device=log_scale.device)
    nd = ctypes.c_int64(0)
    check(lib.pairscreen_build_mask(_ptr(pred) if mode == 0 else None, _ptr(log_scale), n_core, n_h, float(threshold),
                                    float(margin), int(mode), _ptr(mask), ctypes.byref(nd), _ptr(ws),
                                    ctypes.c_size_t(256), _stream(stream)))
    return mask, int(nd.value)

"""Training and application of the learned pair screen through the C ABI.

Orchestration only: every number is computed by libdfpt2.so kernels (plain
pass, pair features, training targets, network training, mask).
"""
from __future__ import annotations

from typing import Iterable

import numpy as np
import torch

from . import api


def collect(inputs: Iterable, s: float, device="cuda"):
    """Features and targets of every core pair of every input set, labelled by the
    plain FP64 pass (its per-pair ||T_ij||_F)."""
    feats, ys = [], []
    for inp in inputs:
        d = api.upload_inputs(inp, device)
        opts = api.make_opts(inp.n_core, inp.n_act, inp.n_vir, inp.n_aux, s)
        r = api.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], want_pair_tnorm=True)
        f, ls = api.pairscreen_features(opts, d["eps_hole"], d["eps_vir"], d["B"])
        y = api.pairscreen_targets(r["pair_tnorm"], ls, inp.n_core, inp.n_h)
        feats.append(f)
        ys.append(y)
    return torch.cat(feats), torch.cat(ys)


def train(feats, y, w0: np.ndarray, steps: int = 1500, lr: float = 3e-3, margin_sigmas: float = 4.0):
    """Full-batch Adam on the GPU.  Returns (weights, losses, margin) with margin =
    margin_sigmas x the root-mean-square training residual (the final loss of the
    kernel's mean squared error); the mask adds it to every predicted log-norm."""
    W = torch.from_numpy(np.asarray(w0, dtype=np.float32)).to(feats.device)
    m = torch.zeros_like(W)
    v = torch.zeros_like(W)
    losses = api.pairscreen_train(W, m, v, feats, y, steps, lr)
    margin = margin_sigmas * float(np.sqrt(max(float(losses[-1].item()), 0.0)))
    return W, losses, margin


def predict_mask(W, opts, eps_hole, eps_vir, B, threshold: float, margin: float, mode: int = 0, stream=None):
    """Screen one input set: (mask [n_h, n_h] uint8 on the device, dropped pairs)."""
    f, ls = api.pairscreen_features(opts, eps_hole, eps_vir, B, stream=stream)
    pred = api.pairscreen_mlp_forward(W, f, stream=stream)[0] if mode == 0 else None
    return api.pairscreen_build_mask(pred, ls, opts.n_core, opts.n_core + opts.n_act, threshold, margin, mode,
                                     stream=stream)

#!/usr/bin/env python3
"""Benchmark of the DF-DSRG-PT2 virtual natural-orbital pass on one MI355X.

Metric: D_vv-build GFLOP/s and ms per pass of the mixed-precision, screened pass
against the plain FP64 pass on the same GPU and inputs, with the energy error
held to 1e-6 Eh.

A step is one pass of the whole hot path over one synthetic input set (inputs
resident in HBM before timing):
    screen   pair features -> network -> mask            (learned pair screening)
    build    dfpt2_build_vv_density (split B into BF16 slices, pair kernel with
             fused DSRG epilogue and energy, density kernel), masked pairs skipped
    fno      fno_truncate (FP64 eigensolver, cumulative-occupation threshold)
    corr     pt2_energy_correction (recanonicalize, transform B, kept-space energy)
value = F_nom / (screen + build time), F_nom = n_aux n_v^2 n_h(n_h+1) + 2 n_h^2 n_v^3,
the same count for every precision (skipped work shows up as speed).
Untimed setup: the screening network is trained on plain-pass labels of 200
small (10 holes, 60 virtuals, 200 aux) input sets, and the plain FP64 pass on the
workload is timed once as the reference the mixed pass is judged against.

    python bench.py [--steps K] [--warmup W] [--workload c4] [--precision int8|bf16|fp8|fp64] [--no-screen]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D_vv build GFLOP/s & ms/pass, mixed+screened vs FP64 at |ΔE|≤1e-6 Eh"
PEAK_TFLOPS = {"f64": 78.6, "bf16": 2500.0, "fp8": 5000.0, "i8": 5000.0}  # dense MFMA (int8: TOP/s)
SCREEN_THRESHOLD = 1e-6

WORKLOADS = {
    # the literal screened workload: c3 sizes, plain generator
    "c4": dict(base="c4", gen=dict()),
    # localized variant of the same sizes (hole/aux positions, xi = 1.25) where pairs decay
    "c4loc": dict(base="c4", gen=dict(localized_xi=1.25)),
    "c3": dict(base="c3", gen=dict()),
    "c2": dict(base="c2", gen=dict(low_rank=64)),
    "c5": dict(base="c5", gen=dict()),
    # the screened variant of the largest one-GPU instance: c5 sizes, localized holes and
    # auxiliary functions (xi = 1.25)
    "c5loc": dict(base="c5", gen=dict(localized_xi=1.25)),
    # c3 sizes with a redundant auxiliary set (rank 2000 of 4000 up to 1e-7 noise): the
    # input natural auxiliary functions compress (--naf-scan)
    "c4naf": dict(base="c4", gen=dict(aux_rank=2000, aux_noise=1e-7)),
}


def nominal_flops(n_h, n_v, n_aux):
    return n_aux * n_v * n_v * n_h * (n_h + 1) + 2 * n_h * n_h * n_v ** 3


def load_golden(workload, s):
    name = {"c4": "c3"}.get(workload, workload)
    path = os.path.join(ROOT, "tests", "golden", f"{name}_s{s:g}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def dd(a, b):
    return abs(math.fsum([a[0], a[1], -b[0], -b[1]]))


def cpu_baseline(inp, s, target_seconds=15.0):
    """The FP64 oracle on the first k core holes of the same workload (full n_v and
    n_aux), k chosen for about target_seconds of work; nominal flops / wall time."""
    from oracle import dsrg_pt2 as o
    import numpy as np
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    nv, na = inp.n_vir, inp.n_aux

    def run(k):
        sub = inp.replace(eps_core=inp.eps_core[:k], eps_act=np.zeros(0), gamma_act=np.zeros((0, 0)),
                          B=np.ascontiguousarray(inp.B[:k]))
        t0 = time.perf_counter()
        o.pt2_pass_inputs(sub, s)
        return time.perf_counter() - t0

    run(1)
    t2 = run(2)
    per_pair = max(t2 / 4.0, 1e-4)
    k = int(max(2, min(inp.n_core, (target_seconds / per_pair) ** 0.5)))
    dt = run(k)
    F = nominal_flops(k, nv, na)
    return {"value": F / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 NumPy oracle pass (energy + D_vv) over the first {k} of {inp.n_core} holes "
                      f"at n_v={nv}, n_aux={na} ({k * k} ordered pairs, {dt:.1f} s); nominal flops / wall time"}


def recorded_traffic(kernel: str, workload: str):
    """HBM-side bytes per launch of `kernel` on `workload` from a committed hardware-counter
    summary under profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter
    reads for a device copy of known size).  None if there is no record, or if the kernel's
    sources have changed since the counters were taken (recorded SHA-256 of the sources)."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if kv.get("kernel") != kernel or kv.get("workload") != workload:
                    continue
                h = hashlib.sha256()
                for src in kv["sources"].split(","):
                    with open(os.path.join(ROOT, src), "rb") as g:
                        h.update(g.read())
                if h.hexdigest() != kv["sha256"]:
                    return None
                return 1024.0 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                                 float(kv["write_kib"]) * float(kv["write_scale"]))
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def active_particle_bench(args, wl, cfg):
    """dfpt2_add_active_particle_density on the workload's sizes (needs n_act > 0)."""
    import torch
    import synth
    import paper_2312_07008_amd as dp

    s = args.s if args.s is not None else cfg["s"][0]
    n_core, n_act, n_v, n_aux = cfg["sizes"]
    if n_act == 0:
        raise SystemExit("--active-particles needs a workload with active orbitals (c2, c5)")
    inp = synth.generate(n_core, n_act, n_v, n_aux, 0, label=args.workload, active_particles=True, **wl["gen"])
    d = dp.upload_inputs(inp)
    del inp
    opts = dp.make_opts(n_core, n_act, n_v, n_aux, s)
    stream = torch.cuda.current_stream()
    D = torch.zeros((n_v, n_v), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        dp.add_active_particle_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], d["B_act"], D)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        dp.add_active_particle_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], d["B_act"], D)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    n_h = n_core + n_act
    K = n_h * n_h * n_act
    flops = 2.0 * n_v * K * n_aux + 2.0 * n_v * K * n_act + 2.0 * n_v * n_v * K
    res = {"metric": "Eq. A9 active-particle terms ms", "value": ms, "unit": "ms", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic", "config": {"workload": f"{args.workload} sizes with active-particle integrals",
                                           "n_core": n_core, "n_act": n_act, "n_vir": n_v, "n_aux": n_aux},
           "gemm_flops": flops, "tflops": flops / (ms * 1e-3) / 1e12,
           "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12, "peak": PEAK_TFLOPS["f64"],
                        "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["f64"],
                        "traffic": None, "kernel": "gemm_f64 (amplitudes, eta, rank update) + mixing kernels"}}
    log(f"active-particle terms: {ms:.2f} ms, {res['tflops']:.1f} TFLOP/s")
    # the singles (Eq. A6) and the two-body-cumulant terms of Eq. A9, with a synthetic cumulant
    lam = torch.from_numpy(synth.active_cumulant(n_act, 0)).cuda()
    ncs = dp.add_cumulant_singles_density
    for _ in range(args.warmup):
        ncs(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], lam, d["B"], d["B_act"], D)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ncs(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], lam, d["B"], d["B_act"], D)
    e1.record(stream)
    torch.cuda.synchronize()
    ms2 = e0.elapsed_time(e1) / args.steps
    kl = 2 * n_h * n_act ** 2 + n_act ** 3 + n_h + 2 * n_act
    f2 = (2.0 * n_v * n_h * n_h * n_act * n_aux + 2.0 * n_v * n_v * n_act * n_act * n_aux
          + 2.0 * n_v * n_act ** 4 * n_v + 2.0 * n_v * n_v * (kl + n_act * n_act * n_v))
    res["cumulant_singles"] = {"ms": ms2, "gemm_flops": f2, "tflops": f2 / (ms2 * 1e-3) / 1e12,
                               "frac_of_f64_peak": f2 / (ms2 * 1e-3) / 1e12 / PEAK_TFLOPS["f64"],
                               "terms": "Eq. A6 singles and the Eq. A9 terms with singles or the two-body cumulant"}
    log(f"singles + cumulant terms: {ms2:.2f} ms, {res['cumulant_singles']['tflops']:.1f} TFLOP/s")
    print(json.dumps(res), flush=True)


def ladder_bench(args, wl, cfg):
    """Particle-particle ladder R^p = sum_cd (ac|bd) T^p_cd at N_V and at N_V' (kept NOs of the
    workload's FP64 pass at p_o): the (N_V/N_V')^4 saving the truncation is for (Sec. 2, Eq. 6)."""
    import numpy as np
    import torch
    import synth
    import paper_2312_07008_amd as dp

    s = args.s if args.s is not None else cfg["s"][0]
    p_o = args.p_o if args.p_o is not None else cfg["p_o"][0]
    n_core, n_act, n_v, n_aux = cfg["sizes"]
    inp = synth.generate(n_core, n_act, n_v, n_aux, 0, label=args.workload, **wl["gen"])
    d = dp.upload_inputs(inp)
    o64 = dp.make_opts(n_core, n_act, n_v, n_aux, s, precision=dp.FP64)
    r = dp.build_vv_density(o64, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"])
    t = dp.fno_truncate(r["D_vv"], p_o)
    k = t["n_kept"]
    del r, d
    torch.cuda.empty_cache()
    n_amp = args.ladder_amps or n_core * n_core
    t0 = time.time()
    lin = synth.ladder_inputs(n_v, n_aux, n_amp, seed=0)
    log(f"ladder inputs n_v={n_v} n_aux={n_aux} n_amp={n_amp} in {time.time() - t0:.1f} s; kept {k} of {n_v}")
    B = torch.from_numpy(lin.B_vv).cuda()
    T = torch.from_numpy(lin.T).cuda()
    del lin
    stream = torch.cuda.current_stream()
    out = {}
    for name, X, m in (("full", None, n_v), ("kept", t["no_vecs"], k)):
        ws = torch.empty(dp.pp_ladder_workspace_size(n_v, n_aux, n_amp, 0 if X is None else m), dtype=torch.uint8,
                         device="cuda")
        R = torch.empty((n_amp, m, m), dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            dp.pp_ladder(B, T, X, m, R=R, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        dp.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            dp.pp_ladder(B, T, X, m, R=R, workspace=ws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        prof = dp.profile_read()
        dp.profile_enable(False)
        ms = e0.elapsed_time(e1) / args.steps
        flops = 2.0 * m ** 4 * (n_aux + n_amp)
        out[name] = {"n_virtual": m, "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                     "transform_ms": prof["ladder_transform"][0] / args.steps,
                     "contraction_ms": prof["ladder"][0] / args.steps}
        log(f"ladder {name}: N={m} {ms:.1f} ms, {out[name]['tflops']:.1f} TFLOP/s")
        del ws, R
        torch.cuda.empty_cache()
    ratio = out["full"]["ms"] / out["kept"]["ms"]
    res = {"metric": "particle-particle ladder ms at N_V and at N_V' (FNO)", "value": ratio,
           "unit": "x (full / kept time)", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{args.workload} sizes, ladder over {n_amp} amplitude matrices, p_o={p_o}",
                      "n_vir": n_v, "n_kept": k, "n_aux": n_aux, "n_amp": n_amp},
           "predicted_ratio": (n_v / k) ** 4, "full": out["full"], "kept": out["kept"],
           "roofline": {"bound": "mfma", "achieved": out["full"]["tflops"], "peak": PEAK_TFLOPS["f64"],
                        "unit": "TFLOP/s", "frac": out["full"]["tflops"] / PEAK_TFLOPS["f64"],
                        "traffic": None, "kernel": "gemm_f64 (ladder integrals + contraction)"}}
    print(json.dumps(res), flush=True)


def screen_gain(W, margin, s, p_o, prec, steps=3):
    """What the learned screen gains on the localized variant of the headline sizes
    (80 core holes, 1200 virtuals, 4000 auxiliary functions; hole and auxiliary
    positions with xi = 1.25, so pair norms span many decades): the screened pass
    (features, network, mask, then the pass on the surviving pairs) against the
    unscreened pass at the same precision, both timed with inputs in HBM, judged by
    the unscreened pass and by the plain FP64 pass on the same inputs."""
    import numpy as np
    import torch
    import synth
    import paper_2312_07008_amd as dp
    from paper_2312_07008_amd import screening

    t0 = time.time()
    inp = synth.generate(80, 0, 1200, 4000, 0, label="c4loc", localized_xi=1.25)
    d = dp.upload_inputs(inp)
    del inp
    log(f"screen gain: c4loc inputs in {time.time() - t0:.1f} s")
    stream = torch.cuda.current_stream()
    n_core, n_v = 80, 1200
    n_up = n_core * (n_core + 1) // 2
    opts = dp.make_opts(80, 0, 1200, 4000, s, precision=prec)
    o64 = dp.make_opts(80, 0, 1200, 4000, s, precision=dp.FP64)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    r64 = dp.build_vv_density(o64, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], want_pair_tnorm=True,
                              stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    fp64_ms = e0.elapsed_time(e1)
    t64 = dp.fno_truncate(r64["D_vv"], p_o)
    E64 = tuple(float(x) for x in r64["e_pt2"].cpu().numpy())
    occ64, tn64 = t64["occ"].cpu().numpy(), r64["pair_tnorm"].cpu().numpy()
    del r64
    torch.cuda.empty_cache()
    ws = torch.empty(dp.workspace_size(opts), dtype=torch.uint8, device="cuda")
    D = torch.empty((n_v, n_v), dtype=torch.float64, device="cuda")
    e = torch.empty(2, dtype=torch.float64, device="cuda")
    out = {}
    for name in ("unscreened", "screened"):
        times, nd, mask = [], 0, None
        for it in range(steps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            if name == "screened":
                mask, nd = screening.predict_mask(W, opts, d["eps_hole"], d["eps_vir"], d["B"], SCREEN_THRESHOLD,
                                                  margin, stream=stream)
            dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], mask, D_vv=D, e_pt2=e,
                                workspace=ws, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            if it:
                times.append(a.elapsed_time(b))
        t = dp.fno_truncate(D, p_o)
        out[name] = dict(ms=statistics.median(times), E=tuple(float(x) for x in e.cpu().numpy()),
                         occ=t["occ"].cpu().numpy(), n_kept=t["n_kept"], nd=nd,
                         mask=None if mask is None else mask.cpu().numpy())
        log(f"screen gain: {name} {out[name]['ms']:.1f} ms per pass, kept {t['n_kept']}, dropped {nd}")
    del ws, D
    torch.cuda.empty_cache()
    u, sc = out["unscreened"], out["screened"]
    mk = sc["mask"]
    dropped = [(i, j) for i in range(n_core) for j in range(i, n_core) if mk[i, j] == 0]
    wrong = sum(1 for i, j in dropped if not tn64[i, j] < SCREEN_THRESHOLD)
    below = sum(1 for i in range(n_core) for j in range(i, n_core) if tn64[i, j] < SCREEN_THRESHOLD)
    return {"workload": "c4loc: 80 core holes, 1200 virtuals, 4000 auxiliary functions, localized holes and "
                        "auxiliary functions (xi = 1.25), seed 0",
            "threshold": SCREEN_THRESHOLD, "pairs_total": n_up, "pairs_dropped": sc["nd"],
            "pairs_dropped_above_threshold_in_fp64_pass": wrong,
            "pairs_below_threshold_in_fp64_pass": below,
            "ms_per_pass_unscreened": u["ms"], "ms_per_pass_screened": sc["ms"],
            "speedup_screened_vs_unscreened": u["ms"] / sc["ms"], "fp64_ms_per_pass": fp64_ms,
            "speedup_screened_vs_fp64": fp64_ms / sc["ms"],
            "delta_E_vs_unscreened_Eh": dd(sc["E"], u["E"]), "delta_E_vs_fp64_Eh": dd(sc["E"], E64),
            "max_dON_vs_unscreened": float(np.abs(sc["occ"] - u["occ"]).max()),
            "max_dON_vs_fp64": float(np.abs(sc["occ"] - occ64).max()),
            "n_kept": {"screened": sc["n_kept"], "unscreened": u["n_kept"], "fp64": t64["n_kept"]}}


def library_gemm_context(n_v, n_aux, batch=64):
    """The vendor library's BF16 GEMM (torch.matmul / bmm on hipBLASLt) timed on this
    part, for context beside the product kernel's fraction: one slice product of a
    batch of pairs at the pass's own shape (n_v x n_v x n_aux) and one large square
    GEMM.  Not part of the pass; contiguous operands only."""
    import torch
    out = []
    for (m, n, k, nb) in ((n_v, n_v, n_aux, batch), (8192, 8192, 8192, 1)):
        a = torch.randn(nb, m, k, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(nb, k, n, device="cuda", dtype=torch.bfloat16)
        f = (lambda: torch.matmul(a[0], b[0])) if nb == 1 else (lambda: torch.bmm(a, b))
        # warm-up of about 100 ms (the clock settles under load), then at least 100 ms timed
        for _ in range(3):
            f()  # the first calls pick and load the library's kernel
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        f()
        ev[1].record()
        torch.cuda.synchronize()
        reps = max(10, int(100.0 / max(ev[0].elapsed_time(ev[1]), 1e-3)))
        for _ in range(reps):
            f()
        ev[0].record()
        for _ in range(reps):
            f()
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        tf = 2.0 * m * n * k * nb / ms / 1e9
        out.append({"m": m, "n": n, "k": k, "batch": nb, "reps": reps, "ms": ms, "TFLOP_s": tf, "frac": tf / PEAK_TFLOPS["bf16"]})
        del a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="bf16", choices=["int8", "bf16", "fp8", "fp64"])
    ap.add_argument("--no-screen", action="store_true")
    ap.add_argument("--slices-gemm2", type=int, default=0,
                    help="slices (BF16) or digits (INT8) per operand of the density product; 0 = library default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-ref", action="store_true")
    ap.add_argument("--s", type=float, default=None)
    ap.add_argument("--p-o", type=float, default=None)
    ap.add_argument("--naf-scan", action="store_true",
                    help="after the timed steps: natural auxiliary functions at several relative thresholds, "
                         "the compression time, n_naf, and the pass time and energy on the compressed integrals")
    ap.add_argument("--no-screen-gain", action="store_true",
                    help="skip the screened-vs-unscreened measurement on the localized workload (c4loc) that a "
                         "default c4 run reports in screen_gain")
    ap.add_argument("--no-library-gemm", action="store_true",
                    help="skip the vendor BF16 GEMM timed beside a BF16 run for context")
    ap.add_argument("--no-alt", action="store_true",
                    help="skip the INT8-digit measurement reported beside a BF16 run")
    ap.add_argument("--ladder", action="store_true",
                    help="instead of the pass: time the particle-particle ladder (the N_V^4 contraction of the "
                         "high-level step) in the full virtual space and in the space of the kept NOs of the "
                         "workload's FP64 pass, and print one JSON line for it")
    ap.add_argument("--active-particles", action="store_true",
                    help="instead of the pass: time dfpt2_add_active_particle_density (the Eq. A9 terms with an "
                         "active particle index) on the workload's sizes, and print one JSON line for it")
    ap.add_argument("--ladder-amps", type=int, default=0,
                    help="amplitude matrices of the ladder run (default: every ordered core pair)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one device-to-device copy of this many MiB before timing (a reference "
                         "kernel of known traffic for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported (the pass would shard hole "
              "pairs over GPUs with one D_vv all-reduce, which is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2312_07008_amd as dp
    from paper_2312_07008_amd import screening

    wl = WORKLOADS[args.workload]
    cfg = synth.CONFIGS[wl["base"]]
    if args.ladder:
        return ladder_bench(args, wl, cfg)
    if args.active_particles:
        return active_particle_bench(args, wl, cfg)
    s = args.s if args.s is not None else cfg["s"][0]
    p_o = args.p_o if args.p_o is not None else cfg["p_o"][0]
    prec = {"fp64": dp.FP64, "bf16": dp.BF16_SLICED, "fp8": dp.FP8_SLICED, "int8": dp.INT8_SLICED}[args.precision]
    dtype = {"fp64": "f64", "bf16": "bf16", "fp8": "fp8", "int8": "i8"}[args.precision]
    screen = not args.no_screen

    t0 = time.time()
    n_core, n_act, n_v, n_aux = cfg["sizes"]
    inp = synth.generate(n_core, n_act, n_v, n_aux, 0, label=args.workload, **wl["gen"])
    log(f"inputs {args.workload} {cfg['sizes']} {wl['gen']} generated in {time.time() - t0:.1f} s")
    d = dp.upload_inputs(inp)
    n_h = inp.n_h
    opts = dp.make_opts(n_core, n_act, n_v, n_aux, s, precision=prec, slices_gemm2=args.slices_gemm2)
    stream = torch.cuda.current_stream()

    # ---- untimed setup: train the screen on small plain-pass labels
    W = None
    margin = 0.0
    train_info = None
    if screen:
        t0 = time.time()
        tr_inputs = (synth.generate(10, 0, 60, 200, seed=k,
                                    localized_xi=(None if k % 2 else 0.6 + 2.4 * ((k * 37) % 97) / 97.0))
                     for k in range(1, 201))
        X, Y = screening.collect(tr_inputs, s)
        W, losses, margin = screening.train(X, Y, synth.mlp_init(0), steps=1500, lr=3e-3)
        torch.cuda.synchronize()
        train_info = {"samples": int(X.shape[0]), "steps": 1500, "final_mse": float(losses[-1].item()),
                      "margin_log": margin, "seconds": time.time() - t0}
        log(f"screen trained on {X.shape[0]} pairs: mse {train_info['final_mse']:.4f}, {train_info['seconds']:.1f} s")

    # ---- untimed reference: the plain FP64 pass on the same inputs
    ref = None
    if not args.no_fp64_ref:
        o64 = dp.make_opts(n_core, n_act, n_v, n_aux, s, precision=dp.FP64)
        ws64 = torch.empty(dp.workspace_size(o64), dtype=torch.uint8, device="cuda")
        times = []
        for it in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            r64 = dp.build_vv_density(o64, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], workspace=ws64,
                                      stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        t64 = dp.fno_truncate(r64["D_vv"], p_o)
        ref = {"ms": min(times), "E": r64["e_pt2"].cpu().numpy(), "occ": t64["occ"].cpu().numpy(),
               "n_kept": t64["n_kept"]}
        del ws64, r64, t64
        torch.cuda.empty_cache()
        log(f"FP64 reference pass {ref['ms']:.1f} ms, kept {ref['n_kept']}")

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {nbytes} bytes done")
        del src, dst

    # the kept-space energy of the correction: INT8 digits after a BF16 or FP8 build (its
    # exact integer sums hold the correction to 1e-6 Eh at the largest sizes, where the
    # BF16 kept-space pass alone is off by ~2e-6 Eh), else the build's own precision
    corr_prec = dp.INT8_SLICED if args.precision in ("bf16", "fp8") else prec
    opts_corr = dp.make_opts(n_core, n_act, n_v, n_aux, s, precision=corr_prec)
    ws_pass = torch.empty(dp.workspace_size(opts), dtype=torch.uint8, device="cuda")
    ws_fno = torch.empty(dp.fno_truncate_workspace_size(n_v), dtype=torch.uint8, device="cuda")
    ws_corr = torch.empty(dp.pt2_correction_workspace_size(opts_corr, n_v), dtype=torch.uint8, device="cuda")
    D = torch.empty((n_v, n_v), dtype=torch.float64, device="cuda")
    e = torch.empty(2, dtype=torch.float64, device="cuda")

    def step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        mask, nd = None, 0
        if screen:
            mask, nd = screening.predict_mask(W, opts, d["eps_hole"], d["eps_vir"], d["B"], SCREEN_THRESHOLD, margin,
                                              stream=stream)
        ev[1].record(stream)
        dp.build_vv_density(opts, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], mask, D_vv=D, e_pt2=e,
                            workspace=ws_pass, stream=stream)
        ev[2].record(stream)
        tr = dp.fno_truncate(D, p_o, workspace=ws_fno, stream=stream)
        ev[3].record(stream)
        c = dp.pt2_energy_correction(opts_corr, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], tr["no_vecs"],
                                     tr["n_kept"], e, workspace=ws_corr, stream=stream)
        ev[4].record(stream)
        return ev, tr, c, nd, mask

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dp.profile_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    records = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof = dp.profile_read()
    dp.profile_enable(False)

    def med(i, j):
        return statistics.median(r[0][i].elapsed_time(r[0][j]) for r in records)

    screen_ms, build_ms, fno_ms, corr_ms = med(0, 1), med(1, 2), med(2, 3), med(3, 4)
    ms_pass = screen_ms + build_ms
    ms_per_step = 1e3 * t_total / args.steps
    F = nominal_flops(n_h, n_v, n_aux)
    value = F / (ms_pass * 1e-3) / 1e9

    # dominant kernel: the pair product V = B_i B_j^T (BF16: its own kernel, the epilogue
    # runs after it; FP8, INT8, FP64: one kernel with the fused epilogue); issued MFMA flops:
    # 2 n_v^2 n_aux per computed unordered core pair and per operand-slice product
    ns1 = {"fp64": 1, "int8": 5}.get(args.precision, 4)
    products = ns1 * (ns1 + 1) // 2
    tr, c, nd, mk = records[-1][1], records[-1][2], records[-1][3], records[-1][4]
    n_up = n_core * (n_core + 1) // 2
    computed = n_up - nd
    # computed pairs i == j: V^{ii} is symmetric, so its algorithmic count is the triangle
    n_diag = n_core if mk is None else int(torch.diagonal(mk)[:n_core].sum().item())
    alg_flops = products * n_aux * (2.0 * n_v * n_v * (computed - n_diag) + n_v * (n_v + 1.0) * n_diag)
    pk_ms, pk_launch = prof["pair"]
    screen_drops = nd > 0  # a different set of launches than the counters were taken on
    achieved = (alg_flops * args.steps) / (pk_ms * 1e-3) / 1e12 if pk_launch else None
    peak = PEAK_TFLOPS[dtype]
    kname = {"int8": "i8"}.get(args.precision, args.precision)
    split_epi = prof["pair_epilogue"][1] > 0
    if split_epi and args.precision == "int8":
        kid, kdesc = f"pair_v_i8_kernel<{ns1},3>", "pair_v_i8 (V = B_i B_j^T, 128 x 128 tiles"
    elif split_epi:
        kid, kdesc = f"pair_v_bf16_kernel<{ns1},4,4>", "pair_v_bf16 (V = B_i B_j^T, 128 x 128 tiles"
    else:
        kid = f"pair_gemm_{kname}_kernel<{ns1},true>"
        kdesc = f"pair_gemm_{kname if ns1 > 1 else 'f64'} (V = B_i B_j^T with the fused DSRG epilogue"
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TOP/s" if dtype == "i8" else "TFLOP/s",
                "frac": (achieved / peak) if achieved else None,
                "traffic": recorded_traffic(kid, args.workload) if (ns1 > 1 and not screen_drops) else None,
                "kernel": f"{kdesc}, {products} slice products)",
                "traffic_unit": "HBM-side bytes per launch: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (factors from a "
                                "1 GiB device copy), from the committed counter summary under profiles/",
                "kernel_ms_per_launch": pk_ms / pk_launch if pk_launch else None,
                "launches_per_pass": pk_launch // args.steps if pk_launch else 0,
                "epilogue_ms_per_launch": (prof["pair_epilogue"][0] / prof["pair_epilogue"][1]) if split_epi else None,
                "flops_per_unit": f"{products} x 2 n_v^2 n_aux per computed unordered core pair i < j, "
                                  f"{products} x n_v (n_v + 1) n_aux per pair i = j (the triangle of the symmetric V^ii)"}

    E = e.cpu().numpy()
    corr = c["correction"].cpu().numpy()
    occ = tr["occ"].cpu().numpy()
    out = {"metric": METRIC, "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": f"{args.workload}: DF-DSRG-PT2 virtual-NO pass, {wl['gen'] or 'plain'} inputs",
                      "n_core": n_core, "n_act": n_act, "n_vir": n_v, "n_aux": n_aux, "s": s, "p_o": p_o,
                      "precision": args.precision, "slices": ns1, "screening": screen,
                      "correction_precision": {dp.FP64: "fp64", dp.BF16_SLICED: "bf16", dp.FP8_SLICED: "fp8",
                                               dp.INT8_SLICED: "int8"}[corr_prec],
                      "screen_threshold": SCREEN_THRESHOLD if screen else None},
           "ms_per_pass": ms_pass,
           "stage_ms_per_step": {"screen": screen_ms, "build": build_ms, "fno_truncate": fno_ms,
                                 "correction": corr_ms},
           "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
           "nominal_gflop_per_pass": F / 1e9, "pairs_dropped": nd, "pairs_total": n_up,
           "n_kept": tr["n_kept"], "margins": list(tr["margins"]),
           "E_pt2": [float(E[0]), float(E[1])], "correction": [float(corr[0]), float(corr[1])],
           "roofline": roofline}
    if train_info:
        out["screen_training"] = train_info
    if args.naf_scan:
        scan = []
        E_full = (float(E[0]), float(E[1]))
        for rel in (1e-10, 1e-8, 1e-6, 1e-4):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            nr = dp.naf_compress(opts, d["B"], rel, stream=stream)
            e1.record(stream)
            k = nr["n_naf"]
            ok = dp.make_opts(n_core, n_act, n_v, k, s, precision=prec)
            rk = dp.build_vv_density(ok, d["eps_hole"], d["eps_vir"], d["gamma_act"], nr["B_naf"].contiguous(),
                                     stream=stream)
            e2.record(stream)
            torch.cuda.synchronize()
            Ek = rk["e_pt2"].cpu().numpy()
            scan.append({"rel_threshold": rel, "n_naf": k, "naf_ms": e0.elapsed_time(e1),
                         "pass_ms": e1.elapsed_time(e2),
                         "delta_E_vs_uncompressed_Eh": dd((float(Ek[0]), float(Ek[1])), E_full)})
            log(f"NAF rel {rel:g}: n_naf {k} of {n_aux}, {scan[-1]['naf_ms']:.0f} ms + pass {scan[-1]['pass_ms']:.0f} ms,"
                f" dE {scan[-1]['delta_E_vs_uncompressed_Eh']:.3e}")
            del nr, rk
            torch.cuda.empty_cache()
        out["naf_scan"] = scan
    if args.precision == "bf16" and not args.no_alt:
        # the same screened build with B as INT8 digits (exact INT32 level sums), untimed by the
        # headline: ms per pass, its pair kernel against the INT8 peak, and its error
        o8 = dp.make_opts(n_core, n_act, n_v, n_aux, s, precision=dp.INT8_SLICED)
        ws8 = torch.empty(dp.workspace_size(o8), dtype=torch.uint8, device="cuda")
        D8 = torch.empty((n_v, n_v), dtype=torch.float64, device="cuda")
        e8 = torch.empty(2, dtype=torch.float64, device="cuda")
        times8 = []
        for it in range(3):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            if it == 1:
                dp.profile_enable(True)
            ev[0].record(stream)
            mask8 = None
            if screen:
                mask8, _ = screening.predict_mask(W, opts, d["eps_hole"], d["eps_vir"], d["B"], SCREEN_THRESHOLD,
                                                  margin, stream=stream)
            dp.build_vv_density(o8, d["eps_hole"], d["eps_vir"], d["gamma_act"], d["B"], mask8, D_vv=D8, e_pt2=e8,
                                workspace=ws8, stream=stream)
            ev[1].record(stream)
            torch.cuda.synchronize()
            if it >= 1:
                times8.append(ev[0].elapsed_time(ev[1]))
        p8 = dp.profile_read()
        dp.profile_enable(False)
        t8 = dp.fno_truncate(D8, p_o)
        E8 = e8.cpu().numpy()
        pk8_ms, pk8_n = p8["pair"]
        ach8 = (15 / products * alg_flops * 2) / (pk8_ms * 1e-3) / 1e12 if pk8_n else None
        out["alt_int8"] = {"ms_per_pass": statistics.median(times8), "n_kept": t8["n_kept"],
                           "pair_kernel_ms_per_launch": pk8_ms / pk8_n if pk8_n else None,
                           "pair_kernel_TOPs": ach8, "pair_kernel_frac_of_int8_peak": ach8 / PEAK_TFLOPS["i8"]
                           if ach8 else None, "E_pt2": [float(E8[0]), float(E8[1])]}
        if ref is not None:
            out["alt_int8"]["delta_E_vs_fp64_Eh"] = dd((float(E8[0]), float(E8[1])),
                                                       (float(ref["E"][0]), float(ref["E"][1])))
            out["alt_int8"]["max_dON_vs_fp64"] = float(np.abs(t8["occ"].cpu().numpy() - ref["occ"]).max())
        log(f"INT8 digits: {out['alt_int8']['ms_per_pass']:.1f} ms per pass, kept {t8['n_kept']}")
        del ws8, D8
        torch.cuda.empty_cache()
    if prec == dp.BF16_SLICED and not args.no_library_gemm:
        try:  # context only: a failure here is recorded and does not stop the line
            out["library_gemm_context"] = library_gemm_context(-(-n_v // 128) * 128, n_aux)
            log("library BF16 GEMM: " + ", ".join(f"{g['m']}x{g['n']}x{g['k']} x{g['batch']} {g['frac']:.3f}"
                                                    for g in out["library_gemm_context"]))
        except RuntimeError as exc:
            out["library_gemm_context"] = {"error": str(exc)[:200]}
            torch.cuda.empty_cache()
    if screen and args.workload == "c4" and not args.no_screen_gain:
        del ws_pass, ws_fno, ws_corr
        torch.cuda.empty_cache()
        out["screen_gain"] = screen_gain(W, margin, s, p_o, prec)
    if ref is not None:
        out["fp64_ms_per_pass"] = ref["ms"]
        out["speedup_vs_fp64"] = ref["ms"] / ms_pass
        out["delta_E_vs_fp64_Eh"] = dd((float(E[0]), float(E[1])), (float(ref["E"][0]), float(ref["E"][1])))
        out["max_dON_vs_fp64"] = float(np.abs(occ - ref["occ"]).max())
        out["n_kept_fp64"] = ref["n_kept"]
    gold = load_golden(args.workload, s)
    if gold is not None:
        out["delta_E_vs_oracle_Eh"] = dd((float(E[0]), float(E[1])), gold["energy"])
        g_tr = [t for t in gold["truncation"] if abs(t["p_o"] - p_o) < 1e-12]
        if g_tr:
            out["n_kept_oracle"] = g_tr[0]["n_kept"]
            out["delta_correction_vs_oracle_Eh"] = dd((float(corr[0]), float(corr[1])), g_tr[0]["correction"])
        out["max_dON_vs_oracle"] = float(np.abs(occ - np.array(gold["occ"])).max())
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(inp, s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: RK4 steps/s of T+Lambda RT-CC3 at the water-trimer size (o=15, v=57).

One step = one RK4 step of the whole right-hand side (T1 transformation, CCSD
T and Lambda parts, the on-the-fly triples, RHS assembly) times four, plus the
dipole (density with its triples terms) of the step's starting state.  Inputs
are seeded synthetic integrals shaped like the paper's water-trimer cc-pVDZ
workload; the amplitudes live in HBM before the timed region starts.

  python bench.py [--steps K] [--warmup W] [--precision fp64|fp32] [--gpus 1]

Prints one JSON line.  --gpus above 1 exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import torch  # noqa: E402  (device memory and streams of the binding)

def progress(msg):
    """One line per finished phase on stderr (the JSON line stays alone on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


METRIC = "RK4 steps/sec (T+Λ RT-CC3) at o=15,v=57; FP32-split vs FP64 at dipole err"
SIZE_NAMES = {(5, 19): "water-monomer", (10, 38): "water-dimer", (15, 57): "water-trimer",
              (25, 95): "water-pentamer"}
PAPER_GPU_DP_TRIMER_STEPS_PER_S = 1.0 / 806.52  # Table 1, GPU-dp, water trimer (P100)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x2": 2500.0}
PRECISIONS = ("fp64", "fp32", "bf16x3", "bf16x2")
# real bf16 products per complex multiply-add: 4 real products times the kept slice pairs
SLICE_PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 6, "bf16x2": 3}
# HBM bytes per launch of the segmented product, from the two counter passes in
# profiles/build_product_trimer_o15_v57_fp64_traffic.md (FETCH_SIZE, WRITE_SIZE,
# scaled by a 1 GiB copy).  Valid only for the sources they were measured on.
MEASURED_TRAFFIC = {
    "fingerprint": {"kernels.hip": "9c486daae4c66131", "triples.cpp": "5a42de20420d12f9"},
    "config": (15, 57, "fp64"),
    "bytes_per_launch": 10.004e9,
}


def _traffic(o: int, v: int, precision: str):
    """The measured traffic if it applies to these sources and this workload, else None."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2407_18947_amd", "csrc")
    for name, want in MEASURED_TRAFFIC["fingerprint"].items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != want:
                return None
    if MEASURED_TRAFFIC["config"] != (o, v, precision):
        return None
    return MEASURED_TRAFFIC["bytes_per_launch"]


def triples_flops_per_step(o: int, v: int) -> float:
    """Algorithmic flops of the triples work in one RK4 step (8 real flops per
    complex multiply-add; each distinct t3/lambda3 element built once).

    Per right-hand side: o^3 v^4 terms: t3 build (1), lambda3 build (2), X2 (1),
    Y2 (1), Y1 via Z_i^{bde} (1); o^4 v^3 terms: t3 (1), lambda3 (2), X2 (1),
    Y2 (1), Y1 intermediates (9).  Per step: four right-hand sides plus the
    density terms D_ab (o^3 v^4) and D_ij, D_ia (3 o^4 v^3).
    """
    a, b = o ** 3 * v ** 4, o ** 4 * v ** 3
    per_rhs = 6 * a + 15 * b
    return 8.0 * (4 * per_rhs + a + 3 * b)


def cpu_baseline(system, y0, E, blocks: int):
    """Time the oracle on a bounded sample and scale it to one RK4 step."""
    import torch

    from oracle import rtcc3 as orc

    m = orc.Model.from_system(system)
    o = m.o
    t0 = time.time()
    orc.rhs_terms(m, y0, E, with_triples=False, with_density=True)
    t_ccsd = time.time() - t0
    with torch.no_grad():
        t1, t2, l1, l2 = orc.unpack(m, y0)
        ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(E)))
        done = min(o ** 3, int(math.ceil(blocks / o)) * o)
        t0 = time.time()
        orc.triples_loop(m, ti, t2, l1, l2, want_density=False, max_blocks=blocks)
        t_a = (time.time() - t0) / done
        t0 = time.time()
        orc.triples_loop(m, ti, t2, l1, l2, want_density=True, max_blocks=blocks)
        t_b = (time.time() - t0) / done
    nb = o ** 3
    per_step = 3 * (t_ccsd + t_a * nb) + (t_ccsd + t_b * nb)
    return {
        "value": 1.0 / per_step,
        "unit": "RK4 steps/s",
        "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": (f"one CCSD-part evaluation plus {done} of {nb} occupied-triple blocks of the oracle's "
                   f"triples loop, timed with and without density terms and scaled to 4 RHS + density "
                   f"= one RK4 step ({per_step:.0f} s/step)"),
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def alpha_proxy(make_ctx, y0, steps, dt, amp, codes, precisions):
    """Polarisability proxy per precision: mu^(1)_z(t) from the four-point central
    finite-field formula (Sec. 2.2.2) over delta kicks of +-amp and +-2 amp along z,
    mu1 = [8 (mu(A) - mu(-A)) - (mu(2A) - mu(-2A))] / (12 A); four propagations of
    `steps` RK4 steps per precision on one context (state reset between them)."""
    from paper_2407_18947_amd import _lib
    from paper_2407_18947_amd.inputs import field_delta_kick

    ctx = make_ctx()
    out = {}
    try:
        for prec in precisions:
            ctx.set_option(_lib.RTCC3_OPT_PRECISION, codes[prec])
            mus = {}
            for k in (1, -1, 2, -2):
                ctx.set_state(y0)
                mus[k] = ctx.propagate(steps, dt, field_delta_kick(steps, dt, k * amp, "z"))[:, 2]
            out[prec] = (8.0 * (mus[1] - mus[-1]) - (mus[2] - mus[-2])) / (12.0 * amp)
    finally:
        ctx.close()
    return out


def derivatives(codes, split, steps, dt=0.025, amp=0.001, h=1e-5, o=10, v=38, seed=2):
    """Derivative of the dipole series with respect to the kick amplitude and a
    scale of the dipole integrals at the water-dimer size (forward mode: the
    state and its derivative propagated together, rtcc3_propagate_tangent), its
    cost against the plain propagation, central differences (h) of plain
    propagations as the check, and the split precision's derivative against
    FP64's.  Context creation is outside the timed calls."""
    import dataclasses

    import numpy as np

    from paper_2407_18947_amd import _lib
    from paper_2407_18947_amd.inputs import field_delta_kick, initial_state, make_system

    s = make_system(o, v, seed=seed)
    y0 = initial_state(s)
    shape = field_delta_kick(steps, dt, 1.0, "z")

    def plain(A=amp, scale=1.0):
        sys_ = s if scale == 1.0 else dataclasses.replace(s, mu=s.mu * scale)
        ctx = _lib.Context(sys_, codes["fp64"])
        ctx.set_state(y0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu = ctx.propagate(steps, dt, A * shape)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        ctx.close()
        progress(f"derivatives: plain propagation A={A} scale={scale}: {t:.2f} s")
        return mu[:, 2], t

    def tangent(prec):
        ctx = _lib.Context(s, codes[prec])
        ctx.set_option(_lib.RTCC3_OPT_TANGENT, 1)
        out = {}
        for name, fdot, kdot in (("A", shape, 0.0), ("kappa", None, 1.0)):
            ctx.set_state(y0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, d = ctx.propagate_tangent(steps, dt, amp * shape, fdot, kdot)
            torch.cuda.synchronize()
            out[name] = (d[:, 2], time.perf_counter() - t0)
            progress(f"derivatives: {prec} d/d{name}: {out[name][1]:.2f} s")
        ctx.close()
        return out

    mu, t_plain = plain()
    fd = {"A": (plain(amp + h)[0] - plain(amp - h)[0]) / (2 * h),
          "kappa": (plain(amp, 1 + h)[0] - plain(amp, 1 - h)[0]) / (2 * h)}
    t64 = tangent("fp64")
    tsp = tangent(split)
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    return {
        "workload": (f"o={o}, v={v}, naux={s.naux}, seed {seed}, delta kick {amp} a.u. along z, "
                     f"{steps} RK4 steps of dt={dt}; d mu_z(t_n)/dA and d mu_z(t_n)/dkappa"),
        "plain_ms_per_step": 1e3 * t_plain / steps,
        "fp64": {p: {"ms_per_step": 1e3 * t64[p][1] / steps, "cost_vs_plain": t64[p][1] / t_plain,
                     "rel_err_vs_central_difference": rel(t64[p][0], fd[p])} for p in ("A", "kappa")},
        split: {p: {"ms_per_step": 1e3 * tsp[p][1] / steps, "cost_vs_plain": tsp[p][1] / t_plain,
                    "rel_err_vs_fp64": rel(tsp[p][0], t64[p][0])} for p in ("A", "kappa")},
        "central_difference_h": h,
    }


MIXED_BATCH = [(5, 19, 30), (5, 36, 31), (10, 38, 32), (10, 72, 33), (5, 19, 34), (5, 36, 35), (10, 38, 36),
               (10, 72, 37)]


def batched_mixed(codes, precision, steps, dt, amp):
    """The mixed-size batch (two systems each of (o,v) = (5,19), (5,36), (10,38), (10,72),
    seeds 30..37), delta kick along z, every member with a captured step graph:
    lockstep batch against the same members propagated one after another."""
    from paper_2407_18947_amd import _lib
    from paper_2407_18947_amd.inputs import field_delta_kick, initial_state, make_system

    systems = [make_system(o, v, seed=sd) for o, v, sd in MIXED_BATCH]
    ctxs = [_lib.Context(s, codes[precision]) for s in systems]
    try:
        for c in ctxs:
            c.set_option(_lib.RTCC3_OPT_GRAPH, 1)
        f = field_delta_kick(steps, dt, amp, "z")
        fields = [f] * len(ctxs)

        def reset():
            for c, s in zip(ctxs, systems):
                c.set_state(initial_state(s))

        reset()
        _lib.rtcc3_propagate_batch([c.ctx for c in ctxs], 1, dt, [f[:3]] * len(ctxs))  # captures the graphs
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _lib.rtcc3_propagate_batch([c.ctx for c in ctxs], steps, dt, fields)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        reset()
        t0 = time.perf_counter()
        for c in ctxs:
            c.propagate(steps, dt, f)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
    finally:
        for c in ctxs:
            c.close()
    n = len(ctxs)
    return {
        "members": [f"({o},{v}) seed {sd}" for o, v, sd in MIXED_BATCH],
        "precision": precision,
        "steps": steps,
        "aggregate_steps_per_s": n * steps / t_batch,
        "one_after_another_steps_per_s": n * steps / t_seq,
        "speedup_vs_one_after_another": t_seq / t_batch,
    }


def graph_gain(codes, steps, dt, amp, o=5, v=19, seed=1):
    """Steps/s of one small system (monomer size) with its step captured as a graph
    against per-kernel launches from the host."""
    from paper_2407_18947_amd import _lib
    from paper_2407_18947_amd.inputs import field_delta_kick, initial_state, make_system

    s = make_system(o, v, seed=seed)
    out = {}
    f = field_delta_kick(steps, dt, amp, "z")
    for graph in (0, 1):
        ctx = _lib.Context(s, codes["fp64"])
        ctx.set_option(_lib.RTCC3_OPT_GRAPH, graph)
        ctx.set_state(initial_state(s))
        ctx.propagate(2, dt, f[:5])
        ctx.set_state(initial_state(s))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.propagate(steps, dt, f)
        torch.cuda.synchronize()
        out["graph" if graph else "launches"] = steps / (time.perf_counter() - t0)
        ctx.close()
    return {"workload": f"o={o}, v={v}, seed {seed}, fp64", "steps": steps,
            "steps_per_s_launches": out["launches"], "steps_per_s_graph": out["graph"],
            "speedup": out["graph"] / out["launches"]}


def batched_finite_field_trimer(codes, precision, steps, dt, window_blocks, s, y0):
    """The twelve-member finite-field set at the trimer size: three directions times
    delta kicks of +-0.001 and +-0.002 a.u., one lockstep batch (window cap per
    member so that all twelve fit); aggregate steps/s and alpha_zz from the four z
    members by the four-point formula."""
    from paper_2407_18947_amd import _lib
    from paper_2407_18947_amd import properties as P
    from paper_2407_18947_amd.inputs import field_delta_kick

    members = [(d, a) for d in "xyz" for a in (0.001, -0.001, 0.002, -0.002)]
    ctxs = []
    try:
        for _ in members:
            c = _lib.Context(s, codes[precision])
            c.set_option(_lib.RTCC3_OPT_WINDOW_BLOCKS, window_blocks)
            ctxs.append(c)
        for c in ctxs:
            c.set_state(y0)
        fields = [field_delta_kick(steps, dt, a, d) for d, a in members]
        progress(f"finite-field batch: {len(ctxs)} contexts created")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mus = _lib.rtcc3_propagate_batch([c.ctx for c in ctxs], steps, dt, fields)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        progress(f"finite-field batch: {steps} steps of {len(ctxs)} members in {t:.2f} s")
        # one member alone with the same window, for the lockstep's gain
        ctxs[0].set_state(y0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctxs[0].propagate(steps, dt, fields[0])
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t0
    finally:
        for c in ctxs:
            c.close()
    z = {a: mus[i][:, 2] for i, (d, a) in enumerate(members) if d == "z"}
    mu1 = P.finite_field_mu1(z[0.001], z[-0.001], z[0.002], z[-0.002], 0.001)
    return {"members": len(members), "precision": precision, "steps": steps, "window_blocks": window_blocks,
            "aggregate_steps_per_s": len(members) * steps / t, "one_member_alone_steps_per_s": steps / t_one,
            "speedup_vs_one_after_another": (len(members) * steps / t) / (steps / t_one),
            "mu1_z_last": complex(mu1[-1]).real}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=PRECISIONS, default="fp64")
    ap.add_argument("--split", choices=PRECISIONS, default="bf16x3",
                    help="reduced-precision triples path timed beside the main run (dipole error against it)")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--o", type=int, default=15)
    ap.add_argument("--v", type=int, default=57)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--cpu-blocks", type=int, default=60, help="oracle blocks timed for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--window-blocks", type=int, default=0,
                    help="cap the triples windows of the main run at this many ordered blocks (0: one window "
                         "from free memory)")
    ap.add_argument("--single-stream", action="store_true",
                    help="every kernel on one stream, one after another (times each kernel alone; not the metric)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (reference kernel for HBM counters)")
    ap.add_argument("--batch-steps", type=int, default=10,
                    help="steps of the mixed-size batch and of the graph comparison (0: skip both)")
    ap.add_argument("--batch-trimer", type=int, default=0,
                    help="steps of the twelve-member finite-field batch at the trimer size (0: skip)")
    ap.add_argument("--tangent-steps", type=int, default=100,
                    help="RK4 steps of the derivative propagations at the water-dimer size (0: skip)")
    ap.add_argument("--alpha-steps", type=int, default=10,
                    help="RK4 steps of each of the eight finite-field propagations of the polarisability proxy "
                         "(0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np

    from paper_2407_18947_amd import _lib
    from paper_2407_18947_amd.inputs import field_delta_kick, initial_state, make_system

    o, v = args.o, args.v
    dt, amp = 0.05, 0.002
    s = make_system(o, v, seed=args.seed)
    y0 = initial_state(s)
    codes = {"fp64": _lib.RTCC3_FP64, "fp32": _lib.RTCC3_FP32, "bf16x3": _lib.RTCC3_BF16X3,
             "bf16x2": _lib.RTCC3_BF16X2}
    K, W = args.steps, args.warmup
    field = field_delta_kick(W + K, dt, amp, "z")
    torch.cuda.set_device(0)

    tune_rows = []

    def run(precision):
        """W warm-up steps, then K timed steps; returns (s, dipole series, timing)."""
        ctx = _lib.Context(s, codes[precision])
        tune_rows.append(_lib.rtcc3_tuning_report(ctx.ctx))
        if args.single_stream:
            ctx.set_option(_lib.RTCC3_OPT_SINGLE_STREAM, 1)
        if args.window_blocks > 0:
            ctx.set_option(_lib.RTCC3_OPT_WINDOW_BLOCKS, args.window_blocks)
        ctx.set_state(y0)
        mu_w = ctx.propagate(W, dt, field[: 2 * W + 1]) if W > 0 else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu = ctx.propagate(K, dt, field[2 * W: 2 * (W + K) + 1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        timing = _lib.rtcc3_last_timing(ctx.ctx)  # HIP events on the context's stream
        ctx.close()
        series = np.concatenate([np.asarray(mu_w), np.asarray(mu)]) if mu_w is not None else np.asarray(mu)
        return t1 - t0, series, timing

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    secs, mu_main, timing = run(args.precision)
    progress(f"main {args.precision}: {K} steps in {secs:.2f} s")
    steps_per_s = K / secs
    tri_ms_per_step = timing[1] / K
    alg = triples_flops_per_step(o, v)
    achieved = alg / (tri_ms_per_step * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision] / SLICE_PRODUCTS[args.precision]
    b_ms, b_launches, b_flop = timing[3], timing[4], timing[5]
    b_achieved = b_flop / (b_ms * 1e-3) / 1e12 if b_ms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "RK4 steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * secs / K,
        "higher_is_better": True,
        "scaling": "weak",
        # the paper's only timing (Table 1) is for real water-trimer integrals on a P100:
        # context, not this workload's baseline
        "vs_baseline": None,
        "context_paper_p100_gpu_dp_ratio": steps_per_s / PAPER_GPU_DP_TRIMER_STEPS_PER_S,
        "dtype": {"fp64": "f64", "fp32": "f32 triples GEMMs, f64 elsewhere",
                  "bf16x3": "bf16x3-split triples build GEMMs, f32 or f64 other triples GEMMs, f64 elsewhere",
                  "bf16x2": "bf16x2-split triples build GEMMs, f32 or f64 other triples GEMMs, f64 elsewhere"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": (f"RT-CC3 T+Lambda, o={o}, v={v}, naux={s.naux}, seeded synthetic "
                         f"{SIZE_NAMES.get((o, v), 'water-cluster')}-sized integrals (seed {args.seed}), "
                         f"delta kick {amp} a.u. along z, dt={dt}"),
            "o": o, "v": v, "naux": s.naux, "precision": args.precision,
            **({"single_stream": True} if args.single_stream else {}),
            # capped triples windows: blocks held at once and their device memory
            **({"window_blocks": args.window_blocks,
                "window_bytes": args.window_blocks * 16 * v * v * (2 * (-(-v // 8) * 8) + o)}
               if args.window_blocks > 0 else {}),
        },
        # Dominant kernel: the segmented store-mode product, launched for a
        # window's t3 blocks, its lambda3 blocks (before symmetrisation) and
        # the S intermediate of Y1.
        "roofline": {
            "bound": "mfma",
            "kernel": "zgemm_seg_f64_kernel<false> (t3, lambda3 and S products)"
            if args.precision == "fp64" else "segmented products (t3, lambda3, S)",
            "achieved": b_achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": b_achieved / peak,
            "traffic": _traffic(o, v, args.precision),
            "launches": int(b_launches),
            "avg_launch_ms": b_ms / max(b_launches, 1),
            "algorithmic_flop_per_launch": b_flop / max(b_launches, 1),
        },
        # The K-split autotuner's choices for the main context (rows: M, N, K, batch,
        # heuristic split, chosen split, heuristic ms, chosen ms).
        "autotune": {
            "products_tuned": int(len(tune_rows[0])),
            "split_changed": int(np.sum(tune_rows[0][:, 4] != tune_rows[0][:, 5])) if len(tune_rows[0]) else 0,
            "ms_heuristic_sum": float(np.sum(tune_rows[0][:, 6])) if len(tune_rows[0]) else 0.0,
            "ms_chosen_sum": float(np.sum(tune_rows[0][:, 7])) if len(tune_rows[0]) else 0.0,
        },
        # All triples kernels of a step together, against the same peak.
        "triples_engine": {
            "achieved": achieved,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "triples_ms_per_step": tri_ms_per_step,
            "algorithmic_flop_per_step": alg,
        },
    }
    if not args.no_split and args.split != args.precision:
        secs_s, mu_s, timing_s = run(args.split)
        progress(f"split {args.split}: {K} steps in {secs_s:.2f} s")
        tri_s = timing_s[1] / K
        out["split"] = {
            "precision": args.split,
            "value": K / secs_s,
            "unit": "RK4 steps/s",
            "ms_per_step": 1e3 * secs_s / K,
            "ratio_vs_main": (K / secs_s) / steps_per_s,
            "max_dipole_err_vs_main": float(np.abs(mu_s - mu_main).max()),
            "triples_ms_per_step": tri_s,
            "triples_tflops_effective": alg / (tri_s * 1e-3) / 1e12,
        }
        if args.alpha_steps > 0:
            mu1 = alpha_proxy(lambda: _lib.Context(s, codes[args.precision]), y0, args.alpha_steps, dt, 0.001, codes,
                              [args.precision, args.split])
            progress("polarisability proxy done")
            ref = mu1[args.precision]
            out["split"]["alpha_proxy"] = {
                "definition": "max_t |mu1_split - mu1_main| / max_t |mu1_main|, mu1 = four-point finite-field "
                              "first-order dipole (delta kicks +-0.001, +-0.002 a.u. along z)",
                "steps": args.alpha_steps,
                "rel_err": float(np.abs(mu1[args.split] - ref).max() / np.abs(ref).max()),
                "max_abs_mu1": float(np.abs(ref).max()),
            }
    if args.batch_steps > 0:
        out["batched"] = {"mixed": batched_mixed(codes, args.split, args.batch_steps, dt, amp),
                          "graph": graph_gain(codes, args.batch_steps, dt, amp)}
        progress("batched and graph runs done")
    if args.tangent_steps > 0:
        out["derivatives"] = derivatives(codes, args.split, args.tangent_steps)
    if args.batch_trimer > 0:
        out.setdefault("batched", {})["finite_field_trimer"] = batched_finite_field_trimer(
            codes, args.split, args.batch_trimer, dt, 1200, s, y0)
    if not args.no_cpu_baseline:
        progress("oracle sample on the host cores")
        cb = cpu_baseline(s, y0, field[0], args.cpu_blocks)
        cb["cpu_model"] = cpu_model()
        cb["nproc"] = os.cpu_count()
        cb["extrapolated"] = True
        out["cpu_baseline"] = cb
        out["vs_oracle"] = steps_per_s / cb["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput benchmark: batched NGDBF decoding on one MI355X.

Default workload (one step = one batch resident in HBM): the batched
multi-code launch of 2^22 received frames, codes N = 96, 1008, 2048 and 4000
in frame proportions 4:2:1:1, Eb/N0 drawn per frame uniformly in 2..5 dB,
each code with its own decoder parameters (Sec. IV-A), all frames decoded by
one graph-captured ngdbf_decode_batch call.  It prints one JSON line with
decoded information Gbit/s (the value), edge updates/s, BER/FER per code, the
same frames decoded by plain per-code launches, per-step latency, the
dominant kernel's roofline position, the single-code headline point (C1008
SM-NGDBF at 3.5 dB), the other benchmark configurations measured in the same
run (the N=96 point, N=4000 SM-NGDBF at 3.5 dB, the high-rate N=2048 code
with float32 and int8 samples, a short serving window) and the CPU oracle's
rate on a sample of every code.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]
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

METRIC = "decoded info Gbit/s + edge-updates/s on 1 MI355X at fixed BER; p50/p99 decode latency"

# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz.  A SIMD issues vector-ALU work in
# 4-clock slots of 64 lanes: one wave64 instruction per slot, or two in one
# slot when both are of the dual-issue kinds (binary32 fma / mul / add and the
# VOP2 forms of mov, and, or, xor, add_u32, lshrrev), and a transcendental
# takes two slots (measured by --workload issue-rates).  The issue ceiling is
# 256 x 4 x 2.4e9 / 4 slots x 64 lanes = 39.32e12 lane slots/s; a launch fills
# SQ_ACTIVE_INST_VALU - SQ_ACTIVE_INST_VALU2 of them (slots any VALU
# instruction was issued in, less those holding a second one).
PEAK_ISSUE_TSLOTS = 256 * 4 * 2.4e9 / 4 * 64 / 1e12
PEAK_HBM_GBS = 8000.0
# LDS ceiling of the method's on-chip exchange (one bank access per edge
# gather, 2 nnz gathers per frame-round, no bit slicing): 256 CUs x 32 banks
# x 2.4 GHz of bank accesses; bit-iterations/s = that / (2 d_v)
LDS_BANK_ACCESSES = 256 * 32 * 2.4e9


def _heur(ebn0: float):
    """Adaptive-threshold SM-NGDBF parameters of Sec. IV-A: theta -0.9,
    eta 0.95, lambda 0.99 below 3.5 dB, 0.97 at 3.5, 0.94 at 4.0, 0.90 from
    4.25 dB; w = 0.75, Y_max = 2.5, smoothing over the last 64 rounds, T = 300."""
    lam = 0.99 if ebn0 < 3.5 else 0.97 if ebn0 < 4.0 else 0.94 if ebn0 < 4.25 else 0.90
    return dict(w=0.75, theta=-0.9, lam=lam, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)


def _plain(t_max: int):
    return dict(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=t_max, smooth_window=0)


# name -> (code, Eb/N0 dB, params, frames, y format, description)
WORKLOADS = {
    "c1008_sm_3.5dB": ("C1008", 3.5, _heur(3.5), 1 << 20, "f32",
                       "SM-NGDBF (adaptive theta, smoothing), (3,6) N=1008, 3.5 dB, T=300"),
    "c1008_plain_3.5dB": ("C1008", 3.5, _plain(300), 1 << 20, "f32",
                          "plain M-NGDBF, (3,6) N=1008, 3.5 dB, T=300"),
    "c4000_sm_3.5dB": ("C4000", 3.5, _heur(3.5), 1 << 20, "f32",
                       "SM-NGDBF, (3,6) N=4000, 3.5 dB, T=300"),
    "c2048_plain_4.5dB_f32": ("C2048", 4.5, dict(w=0.125, theta=-0.7, lam=1.0, eta=0.65, ymax=2.0,
                                                  t_max=300, smooth_window=0), 1 << 21, "f32",
                              "plain M-NGDBF, (6,32) N=2048, 4.5 dB, T=300, float32 y"),
    "c2048_plain_4.5dB_i8": ("C2048", 4.5, dict(w=0.125, theta=-0.7, lam=1.0, eta=0.65, ymax=2.0,
                                                 t_max=300, smooth_window=0), 1 << 21, "i8",
                             "plain M-NGDBF, (6,32) N=2048, 4.5 dB, T=300, int8 y"),
    "c96_plain_4dB": ("C96", 4.0, _plain(100), 10000, "f32",
                      "plain M-NGDBF, (3,6) N=96, 4 dB, T=100 (10,000 frames)"),
    # parameters of the (6,32) code from the successive-approximation search
    "c2048_tuned_4.5dB_f32": ("C2048", 4.5, dict(w=0.162, theta=-0.287, lam=1.0, eta=0.613, ymax=2.0,
                                                  t_max=300, smooth_window=0), 1 << 21, "f32",
                              "plain M-NGDBF, (6,32) N=2048, 4.5 dB, T=300, searched parameters"),
    "c2048_tuned_4.5dB_i8": ("C2048", 4.5, dict(w=0.162, theta=-0.287, lam=1.0, eta=0.613, ymax=2.0,
                                                 t_max=300, smooth_window=0), 1 << 21, "i8",
                             "plain M-NGDBF, (6,32) N=2048, 4.5 dB, T=300, searched parameters, int8 y"),
    # the quantized hardware-oriented decoder of Sec. IV-E / V-A / V-B
    "c1008_q4_reuse_sm_3.5dB": ("C1008", 3.5, dict(w=0.75, theta=-0.7, lam=0.98, eta=0.95, ymax=1.75,
                                                    t_max=300, smooth_window=64, quant_bits=4,
                                                    noise_reuse=1), 1 << 20, "f32",
                                "quantized SM-NGDBF, Q=4, shift-register noise reuse, (3,6) N=1008, "
                                "3.5 dB, T=300"),
    # single-bit S-NGDBF (Step 3a): one flip per round
    "c1008_s_ngdbf_3.5dB": ("C1008", 3.5, dict(w=0.75, theta=-0.6, lam=1.0, eta=1.0, ymax=2.5,
                                                t_max=100, smooth_window=0, variant=1), 1 << 20, "f32",
                            "S-NGDBF (single-bit argmin flip), (3,6) N=1008, 3.5 dB, T=100"),
}
HEADLINE = "c1008_sm_3.5dB"
DEFAULT = "mix4"
# single-code points measured beside the default batch
EXTRA_POINTS = ["c96_plain_4dB", "c4000_sm_3.5dB", "c2048_plain_4.5dB_f32", "c2048_plain_4.5dB_i8"]


def brief(r: dict) -> dict:
    """The figures of a single-code run that the default line carries."""
    keys = ("value", "unit", "ms_per_step", "edge_updates_per_s", "avg_iterations", "ber", "fer",
            "launch_shape", "latency_ms")
    out = {k: r[k] for k in keys if k in r}
    out["config"] = r["config"]["description"] + f", {r['config']['frames']} frames"
    rf = r.get("roofline") or {}
    out["roofline"] = {k: rf.get(k) for k in ("bound", "frac", "hbm_frac", "lds_busy_frac", "lds_method_ratio")}
    return out

# launch shapes (waves per frame, quads per lane, frames per workgroup) for
# workloads whose default shape is slower: the (6,32) code's searched
# parameter set converges in 12-15 rounds, where four waves per frame with
# two quads per lane beat the default two waves with four quads (84.9 against
# 89.2 ms, int8 73.5 against 75.4); the default wins on the long frames of
# the paper's own parameter set (449 against 476 ms) and the mixed batch
WORKLOAD_SHAPES = {"c2048_tuned_4.5dB_f32": (4, 2, 1), "c2048_tuned_4.5dB_i8": (4, 2, 1)}

# Batched multi-code workload: the four codes in frame proportions 4:2:1:1,
# per-frame Eb/N0 uniform in [2, 5] dB, per-code parameters as above
MIX4 = [("C96", 1 << 21, _plain(100)), ("C1008", 1 << 20, _heur(3.5)),
        ("C2048", 1 << 19, dict(w=0.125, theta=-0.7, lam=1.0, eta=0.65, ymax=2.0, t_max=300,
                                smooth_window=0)),
        ("C4000", 1 << 19, _heur(3.5))]


def kernel_sources_digest() -> str:
    """sha256 over the decoder's device sources (what a counter profile was taken of)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("decode.hip", "kernel.h", "noise.h"):
        with open(os.path.join(ROOT, "paper_1402_2773_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_profile(workload: str):
    """Per-launch hardware counters of the workload's decode kernels from the
    committed rocprofv3 profile (instruction classes, copy-calibrated HBM
    bytes, kernel-trace averages), keyed by the kernel sources' hash; None if
    there is none or the kernel has changed since."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sources_sha256") != kernel_sources_digest():
        return None
    return d


def issue_slots(counters: dict):
    """4-clock vector-ALU issue slots a launch filled (each SIMD's slots with
    at least one VALU instruction issued, summed), or None without the issue
    counters."""
    if "SQ_ACTIVE_INST_VALU" not in counters or "SQ_ACTIVE_INST_VALU2" not in counters:
        return None
    return counters["SQ_ACTIVE_INST_VALU"] - counters["SQ_ACTIVE_INST_VALU2"]


def roofline(code, frames: int, yfmt: str, kernel_ms: float, bit_iters: float, counters,
             per_frame_sigma: bool, kernel: str) -> dict:
    """The kernel's position against the vector-ALU issue ceiling (the bound:
    a large decode launch issues in 0.8-0.9 of the SIMDs' issue slots, while
    HBM and LDS stay far below theirs), with the HBM and LDS fractions of the
    method's algorithmic traffic beside it."""
    ks = kernel_ms / 1e3
    alg_bytes = frames * hbm_bytes_per_frame(code, yfmt, per_frame_sigma)
    dv = code.nnz / code.n
    lds_ceiling_bit_iters = LDS_BANK_ACCESSES / (2 * dv)
    r = {"bound": "alu", "kernel": kernel, "kernel_ms": kernel_ms,
         "unit": "T lane-op slots/s (4-clock wave64 issue slots x 64 lanes)",
         "peak": PEAK_ISSUE_TSLOTS, "achieved": None, "frac": None, "traffic": None,
         "traffic_unit": "bytes/launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
         "algorithmic_bytes": alg_bytes, "hbm_achieved_GBs": alg_bytes / ks / 1e9,
         "hbm_frac": alg_bytes / ks / 1e9 / PEAK_HBM_GBS,
         "lds_method_ratio": bit_iters / ks / lds_ceiling_bit_iters,
         "lds_method_what": "bit-iterations/s against 256 CUs x 32 banks x 2.4 GHz / (2 d_v), the "
                            "ceiling of the method's 2 nnz edge gathers per frame-round at one bank "
                            "access each; not executed work (the incremental syndrome update makes far "
                            "fewer LDS accesses), so it can exceed 1",
         "lds_busy_frac": None,
         "lds_busy_what": "SQ_LDS_IDX_ACTIVE / (GRBM_GUI_ACTIVE x 32 CUs per XCD): the fraction of "
                          "the CUs' clocks in which the LDS was busy (committed profile), at most 1"}
    if counters:
        slots = issue_slots(counters)
        if slots is not None:
            r["achieved"] = slots * 64 / ks / 1e12
            r["frac"] = r["achieved"] / PEAK_ISSUE_TSLOTS
            r["dual_issued_fraction"] = 2 * counters["SQ_ACTIVE_INST_VALU2"] / counters["SQ_INSTS_VALU"]
        r["executed_valu_lane_ops_per_s"] = counters["SQ_INSTS_VALU"] * 64 / ks
        r["valu_instructions_per_launch"] = counters["SQ_INSTS_VALU"]
        if counters.get("traffic_bytes") is not None:
            r["traffic"] = counters["traffic_bytes"]
        lds = counters.get("lds") or {}
        if lds.get("SQ_LDS_IDX_ACTIVE") and lds.get("GRBM_GUI_ACTIVE"):
            r["lds_busy_frac"] = lds["SQ_LDS_IDX_ACTIVE"] / (lds["GRBM_GUI_ACTIVE"] * 32)
        r["counters_from"] = counters.get("source")
    return r


def hbm_bytes_per_frame(code, yfmt: str, per_frame_sigma: bool = False) -> int:
    """y in, packed bits + iteration count + converged flag out."""
    sy = 4 if yfmt == "f32" else 1
    return code.n * sy + (code.n + 7) // 8 + 4 + 1 + (4 if per_frame_sigma else 0)


def host_cpu():
    """Host threads available to this process (its CPU affinity, which on a
    shared host is its share of the machine's logical CPUs) and the CPU model
    name."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def oracle_rate(code, y_host, sigma, params, seed, budget_s: float, cores: int):
    """Frames/s of the CPU oracle on a bounded sample (frames in order from
    the first), and the sample it ran."""
    import numpy as np

    import oracle

    p = oracle.Params(**params)
    sig = sigma if np.ndim(sigma) == 0 else np.asarray(sigma, dtype=np.float32)
    n0 = min(len(y_host), 16 * cores)
    t0 = time.perf_counter()
    oracle.decode(code, y_host[:n0], sig if np.ndim(sig) == 0 else sig[:n0], p, seed, threads=cores)
    dt = time.perf_counter() - t0
    n1 = int(min(len(y_host), max(n0, n0 * budget_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    r = oracle.decode(code, y_host[:n1], sig if np.ndim(sig) == 0 else sig[:n1], p, seed, threads=cores)
    dt = time.perf_counter() - t0
    return n1 / dt, n1, dt, float(r.iters.sum())


def cpu_baseline(code, y_host, sigma, params, seed, budget_s: float):
    """The CPU oracle on a bounded sample of the same workload, on every host
    thread available."""
    oracle_build()
    cores, model = host_cpu()
    fps, n1, dt, iters = oracle_rate(code, y_host, sigma, params, seed, budget_s, cores)
    return {"value": fps * code.k_info / 1e9, "unit": "Gbit/s", "cores": cores, "cpu_model": model,
            "host_logical_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"{n1} of the workload's frames (same code, SNR, parameters), {dt:.1f} s on "
                      f"{cores} host threads",
            "edge_updates_per_s": iters * code.nnz / dt}


def oracle_build():
    import oracle

    oracle.build(force=False)


def stats_of(ng, dev_code, out, t_max: int):
    """Device counters of the decoded frames (ngdbf_frame_stats) as a dict."""
    acc = ng.frame_stats(dev_code, out, t_max).cpu().tolist()
    frames = out.bits.shape[0]
    n = dev_code.n
    return {"frames": frames, "avg_iterations": acc[4] / frames, "ber": acc[0] / (frames * n),
            "fer": acc[2] / frames, "undetected": int(acc[3]), "unconverged_frames": int(acc[5]),
            "iterations": int(acc[4])}


def timed_steps(torch, fn, steps: int, warmup: int, stream):
    """W untimed calls, then K timed ones bracketed by synchronisation; wall
    ms per step and the per-step HIP-event times on `stream`."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    return wall, [e0.elapsed_time(e1) for e0, e1 in ev]


def run_mix4(args) -> int:
    """The batched multi-code launch: one graph replay of one
    ngdbf_decode_batch call over the four codes' jobs per step; then the same
    frames as plain per-code launches one after another (each timed with HIP
    events on its stream: the per-kernel times the roofline uses)."""
    import numpy as np
    import torch

    import paper_1402_2773_amd as ng
    from paper_1402_2773_amd import sweep
    from synth import channel, codes

    scale = args.frames / float(1 << 22) if args.frames else 1.0
    stream = torch.cuda.current_stream()
    items = []
    for idx, (name, frames, params) in enumerate(MIX4):
        frames = max(1, int(frames * scale))
        c = codes.named_code(name)
        sig_h = channel.frame_sigmas(frames, 2.0, 5.0, c.rate, seed=300 + idx)
        sig = torch.from_numpy(sig_h).cuda()
        y = ng.channel(c.n, frames, sig, seed=sweep.channel_seed(320 + idx))
        dc = ng.Code.from_ldpc(c)
        p = ng.Params(**params)
        items.append(dict(name=name, c=c, dc=dc, y=y, sig=sig, sig_h=sig_h, p=p, seed=320 + idx,
                          frames=frames, params=params, out=ng.alloc_outputs(dc, frames, "cuda"),
                          out_plain=ng.alloc_outputs(dc, frames, "cuda")))
    torch.cuda.synchronize()

    # batched: one batch call captured into a graph, each code at the launch
    # shape the autotuner picks on a sample of its own frames (or at the
    # library's default shapes with --no-mix-autotune)
    autotune_ms = {}
    fixed = {}  # --mix-shapes C96=1,1,4:C1008=1,4,16 (counter runs: no tuning launches)
    for spec in filter(None, args.mix_shapes.split(":")):
        name, sh = spec.split("=")
        fixed[name] = tuple(int(v) for v in sh.split(","))
    for it in items:
        if it["name"] in fixed:
            ng.ngdbf_code_set_shape(it["dc"].handle, *fixed[it["name"]])
        elif not args.no_mix_autotune:
            # a sample of its own (same code, parameters and Eb/N0 range, other
            # channel and decoder seeds), several times the resident frames
            n_s = min(it["frames"], 1 << 17)
            idx = [m[0] for m in MIX4].index(it["name"])
            sig_s = torch.from_numpy(channel.frame_sigmas(n_s, 2.0, 5.0, it["c"].rate, seed=900 + idx)).cuda()
            y_s = ng.channel(it["c"].n, n_s, sig_s, seed=sweep.channel_seed(920 + idx))
            t0 = time.perf_counter()
            ng.autotune(it["dc"], y_s, sig_s, it["p"], 940 + idx)
            del y_s, sig_s
            autotune_ms[it["name"]] = {"sample_frames": n_s, "wall_ms": (time.perf_counter() - t0) * 1e3,
                                       "sample": "a tuning sample, not frames of the batch: Eb/N0 U[2,5] dB, channel seed "
                                                 f"{920 + idx}, decoder seed {940 + idx}"}
        it["shape"] = list(ng.ngdbf_code_get_shape(it["dc"].handle, it["p"].c(ng.NGDBF_Y_F32)))
    jobs = [ng.job(it["dc"], it["y"], it["sig"], it["p"], it["seed"], it["out"]) for it in items]
    ng.ngdbf_decode_batch(jobs, None)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            ng.ngdbf_decode_batch(jobs, cs)
    torch.cuda.synchronize()
    batch_ms, step_ms = timed_steps(torch, g.replay, args.steps, args.warmup, stream)

    # plain per-code launches of the same frames, each kernel timed on its stream
    per_code_ms = {}
    for it in items:
        def one(it=it):
            ng.decode(it["dc"], it["y"], it["sig"], it["p"], it["seed"], out=it["out_plain"], stream=stream)
        _, ms = timed_steps(torch, one, max(1, args.steps // 2), 1, stream)
        per_code_ms[it["name"]] = float(np.mean(ms))
    plain_ms = sum(per_code_ms.values())

    info_bits = sum(it["frames"] * it["c"].k_info for it in items)
    prof = counter_profile("mix4") if not args.frames else None
    per_code, same = {}, True
    total_iters, total_edges, total_bit_iters = 0, 0.0, 0.0
    for it in items:
        same &= bool(torch.equal(it["out"].bits, it["out_plain"].bits)
                     and torch.equal(it["out"].iters, it["out_plain"].iters))
        st = stats_of(ng, it["dc"], it["out"], it["params"]["t_max"])
        total_iters += st["iterations"]
        total_edges += st["iterations"] * it["c"].nnz
        total_bit_iters += st["iterations"] * it["c"].n
        ms = per_code_ms[it["name"]]
        cnt = prof["instances"].get(it["name"]) if prof else None
        rf = roofline(it["c"], it["frames"], "f32", ms, st["iterations"] * it["c"].n, cnt, True,
                      f"decode_kernel<{','.join(map(str, it['shape'][:2]))},0,false,true,0>")
        per_code[it["name"]] = {**st, "n": it["c"].n, "k": it["c"].k_info, "nnz": it["c"].nnz,
                                "params": it["params"], "shape": it["shape"], "kernel_ms": ms,
                                "info_gbps_plain": it["frames"] * it["c"].k_info / (ms / 1e3) / 1e9,
                                "issue_frac": rf["frac"], "hbm_frac": rf["hbm_frac"],
                                "lds_busy_frac": rf["lds_busy_frac"]}
        if cnt and cnt.get("workgroup_size"):
            # the counters are per kernel instance; frames per workgroup may differ
            per_code[it["name"]]["profiled_workgroup_size"] = int(cnt["workgroup_size"])
            per_code[it["name"]]["workgroup_size"] = 64 * it["shape"][0] * it["shape"][2]
        it["roofline"] = rf
    dominant = max(items, key=lambda it: per_code_ms[it["name"]])
    value = info_bits / (batch_ms / 1e3) / 1e9
    result = {
        "metric": METRIC, "value": value, "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": batch_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded regular LDPC codes, all-zero codeword, BPSK-AWGN from the device "
                "channel (Philox), per-frame Eb/N0 ~ U[2,5] dB",
        "config": {"workload": "mix4", "frames": sum(it["frames"] for it in items),
                   "codes": {it["name"]: it["frames"] for it in items},
                   "ebn0_db": "per frame U[2,5]",
                   "description": "one graph-captured ngdbf_decode_batch of C96:C1008:C2048:C4000 = "
                                  "4:2:1:1 (2^22 frames), per-code parameters (Sec. IV-A)",
                   "autotuned": not args.no_mix_autotune and not fixed,
                   "fixed_shapes": {k: list(v) for k, v in fixed.items()} or None,
                   "autotune": ({"per_code": autotune_ms,
                                 "what": "ngdbf_autotune times every built launch shape (waves per "
                                         "frame, quads per lane, frames per workgroup) that fits the "
                                         "code on the sample and keeps the fastest; untimed"}
                                if autotune_ms else None)},
        "edge_updates_per_s": total_edges / (batch_ms / 1e3),
        "bit_iterations_per_s": total_bit_iters / (batch_ms / 1e3),
        "avg_iterations": total_iters / sum(it["frames"] for it in items),
        "per_code": per_code,
        "plain_per_code_launch": {"ms_per_step": plain_ms, "value": info_bits / (plain_ms / 1e3) / 1e9,
                                  "same_results_as_batched": same},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "what": "one graph replay (the whole mixed batch)"},
        "roofline": {**dominant["roofline"], "code": dominant["name"],
                     "what": "the dominant kernel (longest per-code launch of the mix)"},
    }
    if not args.no_extras:
        result["headline_c1008_sm_3.5dB"] = run_single_point(args, HEADLINE, quiet=True)
        # the other benchmark configurations, measured in the same run: the
        # N=96 point, the N=4000 SM-NGDBF point, the high-rate (6,32) code
        # with float32 and int8 samples (2^21 frames each), and a short
        # serving window (batched runtime only)
        result["other_configs"] = {w: brief(run_single_point(args, w, quiet=True)) for w in EXTRA_POINTS}
        # a parameter-search step as one batch against the same jobs launched
        # one after another
        g = grid_measure(8192, 3, 1)
        result["other_configs"]["grid_c2048_27x8192"] = {
            k: g[k] for k in ("what", "batched_ms", "sequential_ms", "speedup", "batched_info_gbps",
                              "same_results")}
        # (1e4 requests/s of 1-4096 frames offer more frames than one GPU
        # decodes; 2e3/s stays below capacity)
        for rate in (1e4, 2e3):
            srv = serve_measure(rate, 3.0, 4096, True)
            result["other_configs"][f"serve_{int(rate)}_per_s_3s"] = {
                "what": srv["config"]["description"] + f"; Poisson {int(rate)} req/s for 3 s, 1-4096 frames each",
                "info_gbps": srv["batched"]["info_gbps"], "frames_per_s": srv["batched"]["frames_per_s"],
                "latency_ms": srv["batched"]["latency_ms"], "served_requests": srv["batched"]["served_requests"],
                "unserved_requests": srv["batched"]["unserved_requests"], "launches": srv["batched"]["launches"]}
    if not args.no_cpu_baseline:
        oracle_build()
        cores, model = host_cpu()
        cpu_s, sample = 0.0, []
        budget = args.cpu_seconds / len(items)
        for it in items:
            n_h = min(it["frames"], 1 << 14)
            y_h = it["y"][:n_h].cpu().numpy()
            fps, n1, dt, _ = oracle_rate(it["c"], y_h, it["sig_h"][:n_h], it["params"], it["seed"],
                                         budget, cores)
            cpu_s += it["frames"] / fps
            sample.append(f"{it['name']}: {n1} frames in {dt:.1f} s")
        result["cpu_baseline"] = {
            "value": info_bits / cpu_s / 1e9, "unit": "Gbit/s", "cores": cores, "cpu_model": model,
            "host_logical_cpus": os.cpu_count(), "kind": "oracle",
            "sample": "the first frames of every code of the mix (same inputs, parameters, noise keys); "
                      + "; ".join(sample) + f"; whole-mix time extrapolated per code on {cores} host threads"}
    print(json.dumps(result), flush=True)
    for it in items:
        it["dc"].close()
    return 0


def run_serve(args) -> int:
    """Open-loop serving (serve_measure) with the --serve-* options; one JSON line."""
    result = serve_measure(args.serve_rate, args.serve_seconds, args.serve_max_frames,
                           args.serve_batched_only)
    print(json.dumps(result), flush=True)
    return 0


def serve_measure(rate: float, seconds: float, max_frames: int, batched_only: bool) -> dict:
    """Open-loop serving: Poisson request arrivals at `rate` req/s for
    `seconds`, frames per request log-uniform in [1, max_frames], code uniform
    over the four codes, per-request Eb/N0 ~ U[2, 5] dB, decoder seed = request
    id.  The same arrival sequence is served twice by the native runtime:
    continuously batched (every committed request of a code joins one launch)
    and with one launch per request (unless batched_only).  Latency runs from
    a request's scheduled arrival to the host seeing it finished; requests
    still queued when the arrival window closes are reported as unserved."""
    import numpy as np
    import torch

    import paper_1402_2773_amd as ng
    from paper_1402_2773_amd import sweep
    from synth import codes

    names = [name for name, _, _ in MIX4]
    params = [ng.Params(**pr) for _, _, pr in MIX4]
    cl = [codes.named_code(nm) for nm in names]
    dcs = [ng.Code.from_ldpc(c) for c in cl]
    pool = [1 << 18, 1 << 18, 1 << 17, 1 << 16]  # resident slots per code (1 GiB of y at most)
    rng = np.random.default_rng(int(rate) + 17)
    n_req = int(rng.poisson(rate * seconds))
    t_arr = np.sort(rng.uniform(0.0, seconds, n_req))  # Poisson process
    mf = max_frames
    n_fr = np.minimum(np.exp(rng.uniform(0.0, math.log(mf + 1.0), n_req)).astype(np.int64), mf)
    n_fr = np.maximum(n_fr, 1)
    code_of = rng.integers(0, len(names), n_req).astype(np.int32)
    ebn0 = rng.uniform(2.0, 5.0, n_req)
    rates = np.array([c.rate for c in cl])
    sig_req = (1.0 / np.sqrt(2.0 * rates[code_of] * 10.0 ** (ebn0 / 10.0))).astype(np.float32)

    def serve(max_per_launch: int, per_stream: int, window: float):
        srv = ng.Server(dcs, params, pool, n_streams=4, max_requests_per_launch=max_per_launch,
                        launches_per_stream=per_stream)
        queues = [np.nonzero(code_of == c)[0] for c in range(len(names))]
        q_t = [t_arr[q] for q in queues]
        qpos = [0] * len(names)
        # tickets are issued consecutively: ticket -> request through an array
        tick0 = None
        tick2req = np.full(n_req + 16, -1, dtype=np.int64)
        n_live = 0
        t_done = np.full(n_req, np.nan)
        launches = 0
        stream = torch.cuda.current_stream()

        def fill(c, idx, first):
            frames = n_fr[idx]
            tot = int(frames.sum())
            starts = np.repeat(first - np.concatenate(([0], np.cumsum(frames)[:-1])), frames)
            slots = torch.from_numpy(starts + np.arange(tot)).cuda(non_blocking=True)
            sig = torch.from_numpy(np.repeat(sig_req[idx], frames)).cuda(non_blocking=True)
            # the device channel, keyed by the arrival batch's first request
            y = ng.channel(cl[c].n, tot, sig, seed=sweep.channel_seed(int(idx[0]) + 7919))
            srv.pools[c].y.index_copy_(0, slots, y)
            srv.pools[c].sigma.index_copy_(0, slots, sig)

        # warm-up: one request per code, outside the window
        for c in range(len(names)):
            t, first = srv.admit([c], [64], [1 << 40], [0])
            srv.pools[c].y[first[0]:first[0] + 64].fill_(1.0)
            srv.pools[c].sigma[first[0]:first[0] + 64].fill_(0.5)
            srv.commit(t, stream)
        got = 0
        while got < len(names):
            srv.pump()
            d = srv.poll()
            got += len(d)
            srv.release(d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            now = time.perf_counter() - t0
            open_ = now < window
            if open_:
                for c in range(len(names)):
                    q = queues[c]
                    lo = qpos[c]
                    hi = int(np.searchsorted(q_t[c], now, side="right"))
                    if hi <= lo:
                        continue
                    idx = q[lo:min(hi, lo + 65536)]
                    tickets, first = srv.admit(np.full(len(idx), c, np.int32), n_fr[idx], idx.astype(np.uint64),
                                               np.zeros(len(idx), np.uint64))
                    k = len(tickets)
                    if k:
                        fill(c, idx[:k], first)
                        srv.commit(tickets, stream)
                        if tick0 is None:
                            tick0 = int(tickets[0])
                        tick2req[tickets.astype(np.int64) - tick0] = idx[:k]
                        n_live += k
                        qpos[c] += k
            launches += srv.pump()
            done = srv.poll()
            if len(done):
                t_done[tick2req[done.astype(np.int64) - tick0]] = time.perf_counter() - t0
                n_live -= len(done)
                srv.release(done)
            if not open_ and n_live == 0:
                break
        srv.close()
        ok = ~np.isnan(t_done)
        lat = (t_done[ok] - t_arr[ok]) * 1e3
        span = float(np.nanmax(t_done)) if ok.any() else window
        frames_done = int(n_fr[ok].sum())
        info = float(sum(int(n_fr[ok & (code_of == c)].sum()) * cl[c].k_info for c in range(len(names))))
        return {"served_requests": int(ok.sum()), "unserved_requests": int((~ok).sum()),
                "frames": frames_done, "launches": launches,
                "info_gbps": info / span / 1e9, "frames_per_s": frames_done / span,
                "span_s": span,
                "latency_ms": {"p50": float(np.percentile(lat, 50)) if len(lat) else None,
                               "p99": float(np.percentile(lat, 99)) if len(lat) else None,
                               "p99.9": float(np.percentile(lat, 99.9)) if len(lat) else None}}

    batched = serve(32768, 1, seconds)
    print(f"# batched: {batched}", file=sys.stderr, flush=True)
    single = serve(1, 8, seconds) if not batched_only else None
    result = {
        "metric": METRIC, "value": batched["info_gbps"], "unit": "Gbit/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": batched["span_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded regular LDPC codes, all-zero codeword, BPSK-AWGN, Poisson arrivals",
        "config": {"workload": "serve", "rate_req_per_s": rate,
                   "window_s": seconds, "requests": n_req,
                   "frames_per_request": f"log-uniform [1, {mf}]",
                   "offered_frames": int(n_fr.sum()), "codes": names, "pool_slots": pool,
                   "description": "continuous batching over resident slot pools, 4 codes, "
                                  "Eb/N0 ~ U[2,5] dB per request, decoder seed = request id"},
        "latency_ms": batched["latency_ms"], "batched": batched, "per_request_launch": single,
    }
    for d in dcs:
        d.close()
    return result


def run_latency(args) -> int:
    """Per-launch latency of the default workload's decoder for batch sizes
    1 .. 2^16 frames: p50 / p99 of HIP-event times over repeated launches."""
    import numpy as np
    import torch

    import paper_1402_2773_amd as ng
    from paper_1402_2773_amd import sweep
    from synth import channel, codes

    code_name, ebn0, params, _, _, desc = WORKLOADS[HEADLINE]
    code = codes.named_code(code_name)
    sigma = float(np.float32(channel.sigma_from_ebn0(ebn0, code.rate)))
    seed = 2000 + int(round(ebn0 * 10))
    dc = ng.Code.from_ldpc(code)
    p = ng.Params(**params)
    rows = []
    for b in [1, 4, 16, 64, 256, 1024, 4096, 16384, 65536]:
        y = ng.channel(code.n, b, sigma, seed=sweep.channel_seed(seed + b))
        out = ng.alloc_outputs(dc, b, "cuda")
        reps = 200 if b <= 4096 else 50
        stream = torch.cuda.current_stream()
        for _ in range(3):
            ng.decode(dc, y, sigma, p, seed, out=out, stream=stream)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for i, (e0, e1) in enumerate(ev):
            e0.record(stream)
            ng.decode(dc, y, sigma, p, seed, frame_base=i * b, out=out, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
        rows.append({"frames": b, "p50_ms": float(np.percentile(ms, 50)),
                     "p99_ms": float(np.percentile(ms, 99)),
                     "info_gbps_at_p50": b * code.k_info / (np.percentile(ms, 50) / 1e3) / 1e9})
        print(f"# batch {b}: {rows[-1]}", file=sys.stderr, flush=True)
    result = {
        "metric": METRIC, "value": rows[-1]["info_gbps_at_p50"], "unit": "Gbit/s", "n_gpus": 1,
        "steps": len(rows), "warmup": 3, "ms_per_step": rows[-1]["p50_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded (3,6) LDPC code, all-zero codeword, BPSK-AWGN from the device channel",
        "config": {"workload": "latency", "description": desc + "; one launch per batch"},
        "latency_by_batch": rows,
    }
    print(json.dumps(result), flush=True)
    dc.close()
    return 0


def run_single_point(args, workload: str, quiet: bool = False) -> dict:
    """One code at one Eb/N0 (WORKLOADS): K timed launches of the whole batch."""
    import numpy as np
    import torch

    import paper_1402_2773_amd as ng
    from paper_1402_2773_amd import sweep
    from synth import channel, codes

    code_name, ebn0, params, frames, yfmt, desc = WORKLOADS[workload]
    if args.frames and not quiet:
        frames = args.frames
    code = codes.named_code(code_name)
    sigma = float(np.float32(channel.sigma_from_ebn0(ebn0, code.rate)))
    seed = 2000 + int(round(ebn0 * 10))
    dev_code = ng.Code.from_ldpc(code)
    if args.shape and not quiet:
        ng.ngdbf_code_set_shape(dev_code.handle, *[int(v) for v in args.shape.split(",")])
    elif workload in WORKLOAD_SHAPES:
        ng.ngdbf_code_set_shape(dev_code.handle, *WORKLOAD_SHAPES[workload])
    y = ng.channel(code.n, frames, sigma, seed=sweep.channel_seed(seed), int8=yfmt == "i8")
    p = ng.Params(**params)
    out = ng.decode(dev_code, y, sigma, p, seed)  # allocate outputs once
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def step():
        ng.decode(dev_code, y, sigma, p, seed, out=out, stream=stream)

    ms_per_step, step_ms = timed_steps(torch, step, args.steps, args.warmup, stream)
    st = stats_of(ng, dev_code, out, params["t_max"])
    kernel_ms = float(np.mean(step_ms))
    info_gbps = frames * code.k_info / (ms_per_step / 1e3) / 1e9
    prof = (counter_profile(workload)
            if frames == WORKLOADS[workload][3] and not (args.shape and not quiet) else None)
    shape = list(ng.ngdbf_code_get_shape(dev_code.handle, p.c(ng.NGDBF_Y_F32)))
    rf = roofline(code, frames, yfmt, kernel_ms, st["iterations"] * code.n,
                  prof["instances"].get(code_name) if prof else None, False,
                  f"decode_kernel<{shape[0]},{shape[1]},{0 if yfmt == 'f32' else 1},false,true,*>")
    result = {
        "metric": METRIC, "value": info_gbps, "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if yfmt == "f32" else "f32 (int8 y)",
        "data": "synthetic: seeded regular LDPC code, all-zero codeword, BPSK-AWGN from the device channel",
        "config": {"workload": workload, "description": desc, "code": code_name, "n": code.n, "m": code.m,
                   "nnz": code.nnz, "frames": frames, "ebn0_db": ebn0, "sigma": sigma, "params": params,
                   "y_format": yfmt, "seed": seed},
        "edge_updates_per_s": st["iterations"] * code.nnz / (ms_per_step / 1e3),
        "bit_iterations_per_s": st["iterations"] * code.n / (ms_per_step / 1e3),
        "avg_iterations": st["avg_iterations"], "ber": st["ber"], "fer": st["fer"],
        "unconverged_frames": st["unconverged_frames"], "launch_shape": shape,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "what": "one batch launch (all frames of the step)"},
        "roofline": rf,
    }
    # the exact noise skip, counted in one more (untimed) decode: pairs of bits
    # whose decision the radius bound fixed without a Box-Muller transform
    counted = (params.get("variant", 0) == 0 and params.get("quant_bits", 0) == 0
               and params.get("noise_reuse", 0) == 0)
    if counted and not args.no_draw_stats:
        counters = torch.zeros(2, dtype=torch.int64, device="cuda")
        ng.ngdbf_code_set_stats(dev_code.handle, counters)
        ng.decode(dev_code, y, sigma, p, seed, out=out, stream=stream)
        torch.cuda.synchronize()
        ng.ngdbf_code_set_stats(dev_code.handle, None)
        evaluated, transformed = (int(v) for v in counters.cpu().tolist())
        result["gaussian_draws"] = {
            "defined": 2 * evaluated, "transformed": 2 * transformed,
            "skipped_frac": 1.0 - transformed / evaluated if evaluated else None,
            "what": "draws the method defines (one per bit and round) and those the "
                    "kernel computed: the rest could not change a decision"}
    if not args.no_cpu_baseline and not quiet:
        y_host = y[: min(frames, 1 << 16)].cpu().numpy()
        result["cpu_baseline"] = cpu_baseline(code, y_host, sigma, params, seed, args.cpu_seconds)
    dev_code.close()
    del y, out
    return result


def run_phases(args) -> int:
    """Per-round execution counts of the base kernel's data-dependent loops on
    the headline point (C1008 SM-NGDBF, 3.5 dB; one wavefront per frame, lane
    l owning bit quads l, l + 64, l + 128, l + 192), from the decoder's own
    flip traces (ngdbf_decode_trace) and settle-test counters: flips, toggled
    checks, toggle-loop iterations (most flips of one lane), owner-loop
    iterations (most toggles in one 8-check byte of s), the share of rounds
    whose owners apply their events unlisted (more than 64 unsatisfied
    checks at the round's start), u-update passes of the listing rounds
    (events x d_c / 64) and Box-Muller list entries."""
    import numpy as np
    import torch

    import paper_1402_2773_amd as ng
    from paper_1402_2773_amd import sweep
    from synth import channel, codes

    code_name, ebn0, params, _, _, _ = WORKLOADS[HEADLINE]
    if args.ebn0 is not None:
        ebn0, params = args.ebn0, _heur(args.ebn0)
    seed = 2000 + int(round(ebn0 * 10))
    c = codes.named_code(code_name)
    F = args.frames or 1024
    sigma = float(np.float32(channel.sigma_from_ebn0(ebn0, c.rate)))
    y = ng.channel(c.n, F, sigma, seed=sweep.channel_seed(seed))
    dc = ng.Code.from_ldpc(c)
    counters = torch.zeros(2, dtype=torch.int64, device="cuda")
    ng.ngdbf_code_set_stats(dc.handle, counters)
    out = ng.decode(dc, y, sigma, ng.Params(**params), seed, trace=True)
    torch.cuda.synchronize()
    ng.ngdbf_code_set_stats(dc.handle, None)
    Ht = c.dense().astype(np.float32).T
    tr = np.unpackbits(out.trace.cpu().numpy(), axis=-1, bitorder="little")[..., :c.n]
    iters = out.iters.cpu().numpy()
    x0 = (y.cpu().numpy() < 0).astype(np.float32)            # hard-decision errors (all-zero word)
    lane = (np.arange(c.n) // 4) % 64
    sbytes = (c.m + 7) // 8
    dcheck = c.nnz // c.m
    acc = {"flips": [], "toggled_checks": [], "unsatisfied_at_start": [], "toggle_loop_iterations": [],
           "owner_loop_iterations": [], "u_update_iterations": [], "direct": []}
    for f in range(F):
        m = tr[f, : int(iters[f])].astype(np.float32)          # [rounds, n] flips
        if not len(m):
            continue
        tg = (m @ Ht).astype(np.int64) & 1                     # [rounds, m] toggled checks
        xe = (x0[f] + np.vstack([np.zeros((1, c.n), np.float32), np.cumsum(m, 0)[:-1]])) % 2
        unsat = ((xe @ Ht).astype(np.int64) & 1).sum(1)        # unsatisfied checks at each round's start
        per_lane = np.stack([m[:, lane == l].sum(1) for l in range(64)], 1)
        ev = tg.sum(1)
        direct = unsat > 64                                   # rounds whose owners apply events unlisted
        acc["flips"].append(m.sum(1))
        acc["toggled_checks"].append(ev)
        acc["unsatisfied_at_start"].append(unsat)
        acc["toggle_loop_iterations"].append(per_lane.max(1))
        acc["owner_loop_iterations"].append(
            np.pad(tg, ((0, 0), (0, 8 * sbytes - c.m))).reshape(len(tg), sbytes, 8).sum(2).max(1))
        acc["u_update_iterations"].append(np.where(direct, 0, -(-ev * dcheck // 64)))
        acc["direct"].append(direct.astype(np.float64))
    acc = {k: np.concatenate(v) for k, v in acc.items()}
    rounds = int(iters.sum())
    res = {"workload": "phases", "code": code_name, "ebn0_db": ebn0, "frames": F, "rounds": rounds,
           "avg_iterations": rounds / F,
           "per_round": {k: float(np.mean(v)) for k, v in acc.items()},
           "rounds_with_work": float(np.mean(acc["flips"] > 0)),
           "direct_rounds": float(np.mean(acc["direct"])),
           "owner_loop_iterations_per_round_by_kind": {
               "listing": float(np.sum(acc["owner_loop_iterations"] * (1 - acc["direct"])) / len(acc["direct"])),
               "direct": float(np.sum(acc["owner_loop_iterations"] * acc["direct"]) / len(acc["direct"]))},
           "list_entries_per_round": int(counters[1].item()) / rounds,
           "pairs_evaluated_per_round": int(counters[0].item()) / rounds}
    print(json.dumps(res), flush=True)
    dc.close()
    return 0


def run_grid(args) -> int:
    r = grid_measure(args.frames or 8192, args.steps, args.warmup)
    print(json.dumps(r), flush=True)
    return 0 if r["same_results"] else 1


def grid_measure(frames: int, steps: int, warmup: int) -> dict:
    """A parameter-search step as one batch: the (6,32) C2048 code at 4.5 dB,
    27 parameter sets (w, theta, eta each at the searched value and one step
    either side, Sec. IV-A's successive approximation) on the same received
    frames (8192 by default).  The batch runs its jobs concurrently on library
    streams; the same jobs as plain launches run one after another on one
    stream.  Both timed with HIP events; results compared job by job."""
    import numpy as np
    import torch

    import paper_1402_2773_amd as ng
    from paper_1402_2773_amd import sweep
    from synth import channel, codes

    c = codes.named_code("C2048")
    base = sweep.high_rate_tuned_params(4.5)
    sets = [dict(base, w=w, theta=th, eta=eta) for w in (0.14, 0.162, 0.184)
            for th in (-0.25, -0.287, -0.324) for eta in (0.57, 0.613, 0.656)]
    sig = float(np.float32(channel.sigma_from_ebn0(4.5, c.rate)))
    y = ng.channel(c.n, frames, sig, seed=sweep.channel_seed(2048))
    dc = ng.Code.from_ldpc(c)
    ps = [ng.Params(**pr) for pr in sets]
    outs_b = [ng.alloc_outputs(dc, frames, "cuda") for _ in sets]
    outs_s = [ng.alloc_outputs(dc, frames, "cuda") for _ in sets]
    jobs = [ng.job(dc, y, sig, p, 7, o) for p, o in zip(ps, outs_b)]
    stream = torch.cuda.current_stream()

    def batched():
        ng.ngdbf_decode_batch(jobs, stream)

    def sequential():
        for p, o in zip(ps, outs_s):
            ng.decode(dc, y, sig, p, 7, out=o, stream=stream)

    _, b_ms = timed_steps(torch, batched, steps, warmup, stream)
    _, s_ms = timed_steps(torch, sequential, steps, warmup, stream)
    same = all(torch.equal(a.bits, b.bits) and torch.equal(a.iters, b.iters) and
               torch.equal(a.converged, b.converged) for a, b in zip(outs_b, outs_s))
    bm, sm = min(b_ms), min(s_ms)
    info = len(sets) * frames * c.k_info
    r = {
        "workload": "grid", "what": "27 parameter sets of the (6,32) C2048 code at 4.5 dB on the same "
                                    f"{frames} frames (w, theta, eta around the searched set)",
        "jobs": len(sets), "frames_per_job": frames,
        "shape": list(ng.ngdbf_code_get_shape(dc.handle, ps[0].c(ng.NGDBF_Y_F32))),
        "batched_ms": bm, "sequential_ms": sm, "speedup": sm / bm,
        "batched_info_gbps": info / (bm / 1e3) / 1e9, "sequential_info_gbps": info / (sm / 1e3) / 1e9,
        "batched_ms_all": b_ms, "sequential_ms_all": s_ms, "same_results": same}
    dc.close()
    return r


# the issue probe's kinds: one instruction per chain step (kind 1: two)
ISSUE_PROBE_KINDS = [
    "int32 (v_xad_u32)", "int64 product + xor (v_mad_u64_u32, v_xor_b32)", "fp32 fma (v_fmamk_f32)",
    "fp32 mul", "fp32 sqrt (transcendental)", "v_xor_b32", "v_lshlrev_b32", "v_mad_u64_u32",
    "v_bitop3_b32", "v_and_b32", "v_or_b32", "v_mov_b32", "v_cndmask_b32 (VOP3)", "v_add_u32",
    "v_lshrrev_b32", "v_bfe_u32", "v_cmp_eq_u32 (VOP3)", "v_cmp_lt_f32 (VOP3)", "v_readlane_b32",
    "v_writelane_b32", "v_mbcnt_lo_u32_b32", "v_ffbh_u32", "v_lshl_add_u64", "v_add3_u32",
    "v_mad_u32_u24", "v_lshl_add_u32", "v_or3_b32", "v_mul_u32_u24"]


def run_issue_rates(args) -> int:
    """Clocks a wave64 vector-ALU instruction of each class holds its SIMD:
    the library's issue probe (long unrolled chains of one class) at eight
    waves per SIMD, timed with HIP events, at the 2.4 GHz clock."""
    import torch

    import paper_1402_2773_amd as ng

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks, iters = cus * 8, 2000
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    names = ISSUE_PROBE_KINDS
    per_step = [2 if k == 1 else 1 for k in range(len(names))]
    kinds = [int(k) for k in args.probe_kinds.split(",")] if args.probe_kinds else range(len(names))
    rows = []
    for kind in kinds:
        def one(kind=kind):
            ng.ngdbf_issue_probe(kind, blocks, iters, out, stream)
        _, ms = timed_steps(torch, one, 3, 1, stream)
        steps_per_simd = blocks * 4 * iters * 16 * 8 / (cus * 4.0)
        cyc = min(ms) * 1e-3 * 2.4e9 / steps_per_simd / per_step[kind]
        rows.append({"kind": kind, "class": names[kind], "ms": min(ms), "clocks_per_wave64_instruction": cyc})
        print(f"# {rows[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"workload": "issue-rates", "cus": cus, "clock_ghz_assumed": 2.4,
                      "waves_per_simd": 8, "rows": rows}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT,
                    choices=sorted(WORKLOADS) + ["mix4", "serve", "latency", "issue-rates", "phases",
                                                 "grid"])
    ap.add_argument("--frames", type=int, default=0, help="override the batch size")
    ap.add_argument("--ebn0", type=float, default=None,
                    help="phases: Eb/N0 (dB) of the C1008 SM-NGDBF point (default the headline's)")
    ap.add_argument("--shape", default="", help="fix the launch shape: waves,quads,frames_per_block")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="mix4: skip the single-code headline point (profiling runs)")
    ap.add_argument("--no-draw-stats", action="store_true",
                    help="skip the extra decode that counts the Gaussian draws (profiling runs)")
    ap.add_argument("--mix-shapes", default="",
                    help="mix4: fix launch shapes instead of autotuning, e.g. C96=1,1,4:C1008=1,4,16")
    ap.add_argument("--no-mix-autotune", action="store_true",
                    help="mix4: run every code at the library's default shape instead of autotuning it first")
    ap.add_argument("--serve-rate", type=float, default=1e4, help="serve: arrivals per second")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="serve: arrival window")
    ap.add_argument("--serve-max-frames", type=int, default=4096,
                    help="serve: frames per request are log-uniform in [1, this]")
    ap.add_argument("--serve-batched-only", action="store_true")
    ap.add_argument("--probe-kinds", default="", help="issue-rates: comma-separated probe kinds (default all)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this size (for HBM counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the decoder runs on a single MI355X "
              "(frames shard trivially across GPUs, but there is no multi-GPU path). "
              "Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    if args.copy_calibration_mib:
        src_t = torch.ones(args.copy_calibration_mib << 18, dtype=torch.float32, device="cuda")
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
    if args.workload == "mix4":
        return run_mix4(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "latency":
        return run_latency(args)
    if args.workload == "issue-rates":
        return run_issue_rates(args)
    if args.workload == "phases":
        return run_phases(args)
    if args.workload == "grid":
        return run_grid(args)
    print(json.dumps(run_single_point(args, args.workload)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

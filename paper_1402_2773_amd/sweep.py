"""Parameter sweeps and the successive-approximation search of Sec. IV-A.

Every decode goes through the library (one launch per point, or one batched
launch over many parameter sets sharing the same received frames); only the
error counting happens here, on the device, against the all-zero codeword
that the synthetic channel transmits.

  python -m paper_1402_2773_amd.sweep ebn0 --code C1008 --params sm --ebn0 2:5:0.5
  python -m paper_1402_2773_amd.sweep vary --code C1008 --params sm --ebn0 3.5 --vary theta=-1.2:-0.2:0.1
  python -m paper_1402_2773_amd.sweep search --code C2048 --params c2048 --ebn0 4.5
  python -m paper_1402_2773_amd.sweep convergence --code C1008 --ebn0 5 --frames 100
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional, Sequence

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1402_2773_amd as ng  # noqa: E402


def heuristic_params(ebn0: float) -> Dict:
    """SM-NGDBF of Sec. IV-A: theta = -0.9, eta = 0.95, lambda by Eb/N0 (0.99
    below 3.5 dB, 0.97 at 3.5, 0.94 at 4.0, 0.90 from 4.25 dB: the paper's
    setting at 4.25 and 4.5 dB, extended to higher SNR), w = 0.75,
    smoothing over the last 64 rounds, T = 300."""
    lam = 0.99 if ebn0 < 3.5 else 0.97 if ebn0 < 4.0 else 0.94 if ebn0 < 4.25 else 0.90
    return dict(w=0.75, theta=-0.9, lam=lam, eta=0.95, ymax=2.5, t_max=300, smooth_window=64)


def plain_params(ebn0: float) -> Dict:
    """Non-adaptive M-NGDBF: theta = -0.6, eta = 0.9, w = 0.75, T = 300."""
    return dict(w=0.75, theta=-0.6, lam=1.0, eta=0.9, ymax=2.5, t_max=300, smooth_window=0)


def high_rate_params(ebn0: float) -> Dict:
    """The (6,32) code's set: theta = -0.7, eta = 0.65, Y_max = 2.0 (the
    paper's high-rate values), w = 0.125 (w d_v = 0.75), T = 300."""
    return dict(w=0.125, theta=-0.7, lam=1.0, eta=0.65, ymax=2.0, t_max=300, smooth_window=0)


def high_rate_tuned_params(ebn0: float) -> Dict:
    """The (6,32) code's parameters found by successive_approximation at
    4.5 dB on 2^16 frames (from the high-rate set above): w = 0.162,
    theta = -0.287, eta = 0.613, lambda = 1, Y_max = 2.0, T = 300."""
    return dict(w=0.162, theta=-0.287, lam=1.0, eta=0.613, ymax=2.0, t_max=300, smooth_window=0)


PARAM_SETS = {"sm": heuristic_params, "plain": plain_params, "c2048": high_rate_params,
              "c2048t": high_rate_tuned_params}


@dataclasses.dataclass
class Point:
    code: str
    ebn0: float
    params: Dict
    frames: int
    y_format: str
    ber: float
    fer: float
    avg_iterations: float
    unconverged: int
    kernel_ms: float
    info_gbps: float
    seed: int
    fer_ci95: tuple = (0.0, 0.0)        # Wilson interval of the frame error rate
    undetected: int = 0                 # converged to a wrong codeword
    iter_percentiles: tuple = ()        # iterations at p50 / p90 / p99 / max

    def row(self) -> Dict:
        return dataclasses.asdict(self)


def wilson(k: int, n: int, z: float = 1.96):
    """Wilson score interval for k errors in n frames."""
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def _stats(torch, code, out, frames: int, t_max: int, dev_code=None):
    """BER, FER, its interval, undetected errors and iteration percentiles,
    from the device counters of ngdbf_frame_stats (errors against the
    all-zero codeword the synthetic channel sends)."""
    acc = ng.frame_stats(dev_code, out, t_max).cpu().tolist()
    return _from_counters(acc, frames, code.n, t_max)


def _from_counters(acc, frames: int, n: int, t_max: int):
    hist = acc[6:6 + t_max + 1]
    cum, pct, targets = 0, [], [0.5, 0.9, 0.99]
    for t, h in enumerate(hist):
        cum += h
        while targets and cum >= targets[0] * frames:
            pct.append(float(t))
            targets.pop(0)
    top = max((t for t, h in enumerate(hist) if h), default=0)
    fe = int(acc[2])
    return dict(ber=acc[0] / (frames * n), fer=fe / frames, fer_ci95=wilson(fe, frames),
                undetected=int(acc[3]), avg_iterations=acc[4] / frames, unconverged=int(acc[5]),
                iter_percentiles=tuple(pct + [float(top)]))


def _channel(code, ebn0: float, frames: int, seed: int, y_format: str, frame_base: int = 0):
    """Received frames from the device channel (ngdbf_channel), keyed by the
    channel seed and the frames' global indices."""
    import numpy as np

    from synth import channel

    sigma = float(np.float32(channel.sigma_from_ebn0(ebn0, code.rate)))
    y = ng.channel(code.n, frames, sigma, seed=channel_seed(seed), frame_base=frame_base,
                   int8=y_format == "i8")
    return y, sigma


def channel_seed(seed: int) -> int:
    """The channel's Philox key for a run whose decoder key is seed."""
    return (seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) & 0xFFFFFFFFFFFFFFFF


def run_point(code, dev_code, ebn0: float, params: Dict, frames: int, seed: int,
              y_format: str = "f32", y=None, sigma=None) -> Point:
    """Decode `frames` frames at one Eb/N0 and count errors."""
    import torch

    if y is None:
        y, sigma = _channel(code, ebn0, frames, seed, y_format)
    p = ng.Params(**params)
    out = ng.alloc_outputs(dev_code, frames, y.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    ng.decode(dev_code, y, sigma, p, seed, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return Point(code=code.name, ebn0=ebn0, params=params, frames=frames, y_format=y_format,
                 kernel_ms=ms, info_gbps=frames * code.k_info / (ms / 1e3) / 1e9, seed=seed,
                 **_stats(torch, code, out, frames, params["t_max"], dev_code))


def run_point_chunked(code, dev_code, ebn0: float, params: Dict, frames: int, seed: int,
                      chunk: int, state_path: str, y_format: str = "f32",
                      max_chunks: Optional[int] = None) -> Optional[Dict]:
    """A Monte Carlo point in chunks of `chunk` frames with a JSON checkpoint
    after each chunk.  Chunk c decodes frames c*chunk ... with frame_base =
    c*chunk (the noise key) and samples drawn from seed (seed, c), so a run
    resumed from its checkpoint gives bit-identical totals.  Returns the
    totals when every chunk is done, else None (stopped after max_chunks)."""
    import numpy as np
    import torch

    from synth import channel

    n_chunks = (frames + chunk - 1) // chunk
    key = {"code": code.name, "code_digest": code.digest(), "ebn0": ebn0, "params": params,
           "frames": frames, "chunk": chunk, "seed": seed, "y_format": y_format,
           "channel": "device Philox, iteration word 0xFFFFFFFE"}
    state = {"key": key, "next_chunk": 0, "bit_errors": 0, "frame_errors": 0, "undetected": 0,
             "unconverged": 0, "iterations": 0, "iteration_histogram": [0] * (params["t_max"] + 1)}
    if os.path.exists(state_path):
        with open(state_path) as f:
            old = json.load(f)
        if old.get("key") != key:
            raise ValueError(f"{state_path} holds a different run")
        state = old
    sigma = float(np.float32(channel.sigma_from_ebn0(ebn0, code.rate)))
    p = ng.Params(**params)
    done = 0
    while state["next_chunk"] < n_chunks:
        if max_chunks is not None and done >= max_chunks:
            return None
        c = state["next_chunk"]
        fc = min(chunk, frames - c * chunk)
        y = ng.channel(code.n, fc, sigma, seed=channel_seed(seed), frame_base=c * chunk,
                       int8=y_format == "i8")
        out = ng.decode(dev_code, y, sigma, p, seed, frame_base=c * chunk)
        acc = ng.frame_stats(dev_code, out, params["t_max"]).cpu().tolist()
        state["bit_errors"] += int(acc[0])
        state["frame_errors"] += int(acc[2])
        state["undetected"] += int(acc[3])
        state["unconverged"] += int(acc[5])
        state["iterations"] += int(acc[4])
        state["iteration_histogram"] = [a + int(b) for a, b in
                                        zip(state["iteration_histogram"], acc[6:])]
        state["next_chunk"] = c + 1
        tmp = state_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(state, f)
        os.replace(tmp, state_path)
        done += 1
    fe = state["frame_errors"]
    return {**key, "ber": state["bit_errors"] / (frames * code.n), "fer": fe / frames,
            "fer_ci95": wilson(fe, frames), "undetected": state["undetected"],
            "unconverged": state["unconverged"], "avg_iterations": state["iterations"] / frames,
            "iteration_histogram": state["iteration_histogram"]}


def run_grid(code, dev_code, ebn0: float, param_list: Sequence[Dict], frames: int, seed: int,
             y_format: str = "f32") -> List[Point]:
    """Many parameter sets on the same received frames, as one batched launch
    (ngdbf_decode_batch: the jobs run concurrently on library streams)."""
    import torch

    y, sigma = _channel(code, ebn0, frames, seed, y_format)
    outs = [ng.alloc_outputs(dev_code, frames, y.device) for _ in param_list]
    jobs = [ng.job(dev_code, y, sigma, ng.Params(**pr), seed, o) for pr, o in zip(param_list, outs)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    ng.ngdbf_decode_batch(jobs, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(len(param_list), 1)
    pts = []
    for pr, out in zip(param_list, outs):
        pts.append(Point(code=code.name, ebn0=ebn0, params=dict(pr), frames=frames,
                         y_format=y_format, kernel_ms=ms,
                         info_gbps=frames * code.k_info / (ms / 1e3) / 1e9, seed=seed,
                         **_stats(torch, code, out, frames, pr["t_max"], dev_code)))
    return pts


def _score(pt: Point):
    # lower BER first; equal BER (e.g. zero errors): fewer iterations
    return (pt.ber, pt.avg_iterations)


def successive_approximation(code, dev_code, ebn0: float, start: Dict, ranges: Dict[str, tuple],
                             frames: int, seed: int, points: int = 7, shrink: float = 0.35,
                             steps: int = 3, passes: int = 1, log=None) -> Dict:
    """Sec. IV-A: optimise theta, lambda, eta and w one at a time, holding the
    others fixed; each free parameter is searched on a grid over its domain,
    the domain shrinks around the best value, and the search repeats until
    the step is small.  Every grid is one batched launch on the same frames."""
    cur = dict(start)
    for _ in range(passes):
        for name, (lo, hi) in ranges.items():
            a, b = lo, hi
            for _ in range(steps):
                vals = [a + (b - a) * i / (points - 1) for i in range(points)]
                grid = [{**cur, name: v} for v in vals]
                pts = run_grid(code, dev_code, ebn0, grid, frames, seed)
                best = min(pts, key=_score)
                cur[name] = best.params[name]
                if log:
                    log({"search": name, "values": vals, "ber": [p.ber for p in pts],
                         "avg_iterations": [p.avg_iterations for p in pts], "best": cur[name]})
                half = (b - a) * shrink / 2
                a, b = max(lo, cur[name] - half), min(hi, cur[name] + half)
    return cur


# Sec. VI: the decoders compared by average convergence error, T = 100
CONVERGENCE_SET = {
    "S-GDBF": dict(w=1.0, theta=-0.6, lam=1.0, eta=0.0, ymax=2.5, t_max=100, variant=1),
    "M-GDBF (mode switching)": dict(w=1.0, theta=-0.6, lam=1.0, eta=0.0, ymax=2.5, t_max=100,
                                    variant=2),
    "AT-GDBF": dict(w=1.0, theta=-0.6, lam=0.99, eta=0.0, ymax=2.5, t_max=100),
    "S-NGDBF": dict(w=0.75, theta=-0.6, lam=1.0, eta=1.0, ymax=2.5, t_max=100, variant=1),
    "M-NGDBF (adaptive)": dict(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=100),
    "SM-NGDBF": dict(w=0.75, theta=-0.9, lam=0.99, eta=0.95, ymax=2.5, t_max=100,
                     smooth_window=64),
}


def convergence_error(code, dev_code, ebn0: float, params: Dict, frames: int, seed: int) -> Dict:
    """Sec. VI: eps = mean over frames of f(x(T)) - f_max, with f the objective
    of Sec. III-B evaluated by the library (ngdbf_objective) for the decoded
    word and for the sent (all-zero) codeword."""
    import torch

    y, sigma = _channel(code, ebn0, frames, seed, "f32")
    out = ng.decode(dev_code, y, sigma, ng.Params(**params), seed)
    f_out = ng.objective(dev_code, y, params["ymax"], out.bits)
    f_max = ng.objective(dev_code, y, params["ymax"], torch.zeros_like(out.bits))
    torch.cuda.synchronize()
    gap = (f_out - f_max).cpu().numpy().astype("float64") / 2.0 ** 20
    acc = ng.frame_stats(dev_code, out, params["t_max"]).cpu().tolist()
    return {"code": code.name, "ebn0": ebn0, "frames": frames, "params": params,
            "eps": float(gap.mean()), "eps_std": float(gap.std(ddof=1)) if frames > 1 else 0.0,
            "fer": acc[2] / frames, "avg_iterations": acc[4] / frames, "seed": seed}


def _range(spec: str) -> List[float]:
    if ":" not in spec:
        return [float(v) for v in spec.split(",")]
    lo, hi, step = (float(v) for v in spec.split(":"))
    n = int(math.floor((hi - lo) / step + 1e-9)) + 1
    return [round(lo + i * step, 10) for i in range(n)]


def main(argv: Optional[Sequence[str]] = None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("mode", choices=["ebn0", "vary", "search", "convergence"])
    ap.add_argument("--code", default="C1008")
    ap.add_argument("--params", default="sm", choices=sorted(PARAM_SETS))
    ap.add_argument("--set", action="append", default=[], help="override, e.g. t_max=100")
    ap.add_argument("--ebn0", default="3.5")
    ap.add_argument("--frames", type=int, default=1 << 20)
    ap.add_argument("--y-format", default="f32", choices=["f32", "i8"])
    ap.add_argument("--vary", default="", help="name=lo:hi:step (vary mode)")
    ap.add_argument("--seed", type=int, default=0, help="0: 2000 + 10 * Eb/N0")
    ap.add_argument("--out", default="", help="append JSON lines here (default stdout)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="ebn0 mode: frames per chunk, checkpointed to --state (resumable)")
    ap.add_argument("--state", default="", help="checkpoint file prefix for --chunk")
    args = ap.parse_args(argv)

    import torch

    from synth import codes

    if not torch.cuda.is_available():
        print("the sweep needs a HIP device", file=sys.stderr)
        return 1
    code = codes.named_code(args.code)
    dc = ng.Code.from_ldpc(code)
    sink = open(args.out, "a") if args.out else sys.stdout

    def emit(d):
        sink.write(json.dumps(d) + "\n")
        sink.flush()

    def params_at(e):
        pr = PARAM_SETS[args.params](e)
        for kv in args.set:
            k, v = kv.split("=")
            pr[k] = type(pr.get(k, 0.0))(float(v)) if k in pr else int(v)
        return pr

    t0 = time.time()
    for e in _range(args.ebn0):
        seed = args.seed or int(2000 + round(10 * e))
        if args.mode == "ebn0" and args.chunk:
            path = f"{args.state or 'sweep_state'}_{code.name}_{e}.json"
            emit(run_point_chunked(code, dc, e, params_at(e), args.frames, seed, args.chunk, path,
                                   args.y_format))
        elif args.mode == "ebn0":
            emit(run_point(code, dc, e, params_at(e), args.frames, seed, args.y_format).row())
        elif args.mode == "vary":
            name, spec = args.vary.split("=")
            grid = [{**params_at(e), name: v} for v in _range(spec)]
            for pt in run_grid(code, dc, e, grid, args.frames, seed, args.y_format):
                emit(pt.row())
        elif args.mode == "convergence":
            for name, pr in CONVERGENCE_SET.items():
                emit({"algorithm": name, **convergence_error(code, dc, e, pr, args.frames, seed)})
        else:
            ranges = {"theta": (-1.5, -0.1), "lam": (0.85, 1.0), "eta": (0.3, 1.3), "w": (0.05, 1.5)}
            best = successive_approximation(code, dc, e, params_at(e), ranges, args.frames, seed,
                                            log=emit)
            emit({"code": code.name, "ebn0": e, "best_params": best})
            emit(run_point(code, dc, e, best, args.frames, seed + 1, args.y_format).row())
    print(f"# sweep done in {time.time() - t0:.1f} s", file=sys.stderr)
    dc.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Benchmark of the block transform on one MI355X.

A step is one forward transform plus one adjoint transform of a full batch of
the standard GPU workload (4096 blocks, K = 128, M = 15, N = 1920, seeded
16-QAM symbols, shared root-raised-cosine filter with roll-off 0.1), inputs
resident in HBM.  The timed region rotates through several input/output
buffer sets whose total footprint exceeds the GPU's last-level cache, so every
step streams from HBM.

Prints one JSON line: blocks/s over forward + adjoint, the roofline of the
dominant (forward) kernel from HIP events recorded around its launches in the
timed region, the unfused plain-FP32 path and torch.fft (rocFFT) on the same
batch for comparison, the error against the FP64 oracle, and the oracle itself
timed on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "blocks/s and % of HBM/MFMA peak, fwd+adjoint, vs plain FP32 at stated error"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("bt_fused.hpp", "bt_dft.hpp")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1604_06236_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name: str, launch_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (null otherwise)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        e = d[name]
        if e.get("kernel_hash") != kernel_hash():
            return None
        return float(e["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nbuf", type=int, default=4, help="rotating buffer sets")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip plain/rocFFT comparison runs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the block transform has no "
                                   "cross-GPU step (blocks shard by index with no exchange)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1604_06236_amd import transform as T
    from paper_1604_06236_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = W.CONFIGS["plain_gpu"]
    K, M, B = cfg.K, cfg.M, cfg.nblocks
    N = K * M
    S_h, taps_h = W.make_uniform(cfg)
    rng = np.random.default_rng(1234)
    taps = torch.from_numpy(taps_h).to(dev)
    sets = []
    for i in range(args.nbuf):
        S = torch.from_numpy(S_h).to(dev) if i == 0 else torch.from_numpy(
            W.qam(rng, 16, (B, N)).astype(np.complex64)).to(dev)
        yb = torch.from_numpy(W.cn01(rng, (B, N)).astype(np.complex64)).to(dev)
        sets.append((S, torch.empty_like(S), yb, torch.empty_like(S)))
    T.transform_prepare(K, M)
    T.transform_prepare(K, M, "plain_fp32")

    def step(i, ev=None):
        S, y, yb, sb = sets[i % len(sets)]
        if ev is not None:
            ev[0].record()
        T.transform_forward(S, taps, K, M, out=y)
        if ev is not None:
            ev[1].record()
        T.transform_adjoint(yb, taps, K, M, out=sb)
        if ev is not None:
            ev[2].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    adj_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    ms_per_step = wall * 1e3 / args.steps
    blocks_per_s = B / (ms_per_step * 1e-3)

    # roofline of the forward kernel: algorithmic bytes = read S (8N) + write y (8N) per
    # block, plus the shared taps (4N) once per launch
    fwd_bytes = B * 16.0 * N + 4.0 * N
    achieved = fwd_bytes / (fwd_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("fused_forward_128x15", fwd_bytes),
                "kernel": "fused_kernel<Radices<15,16,8>,128,2> (forward)",
                "kernel_ms": round(fwd_ms, 5), "adjoint_kernel_ms": round(adj_ms, 5),
                "algorithmic_bytes_per_launch": fwd_bytes}

    # error against the oracle on a seeded sample of blocks of the timed data
    from oracle import oracle as O
    S0, y0, yb0, sb0 = sets[0]
    step(0)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(0).choice(B, 48, replace=False))
    yh = y0.cpu().numpy()[idx]
    sbh = sb0.cpu().numpy()[idx]
    y_ref = O.forward(S0.cpu().numpy()[idx], taps_h)
    sb_ref, _ = O.adjoint(yb0.cpu().numpy()[idx], taps_h)

    def rel(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    error = {"rel_l2_forward": rel(yh, y_ref), "rel_l2_adjoint": rel(sbh, sb_ref),
             "tolerance": 1e-5, "blocks_checked": int(idx.size)}

    out = {"metric": METRIC, "value": round(blocks_per_s, 1), "unit": "blocks/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded 16-QAM symbols, RRC roll-off 0.1 filter)",
           "config": {"workload": "plain_gpu: 4096 blocks x (K=128, M=15, N=1920), forward + adjoint",
                      "blocks": B, "K": K, "M": M, "N": N, "taps": "shared",
                      "buffer_sets": args.nbuf},
           "roofline": roofline, "error": error}

    if not args.no_compare:
        out["compare"] = compare(T, sets, taps, K, M, B, blocks_per_s, args)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(S_h, taps_h, args.cpu_seconds)

    print(json.dumps(out), flush=True)


def compare(T, sets, taps, K, M, B, blocks_per_s, args):
    """Same batch through the unfused plain-FP32 path and through torch.fft (rocFFT)."""
    import torch
    N = K * M
    res = {}
    ws = torch.empty(T.workspace_size(B, K, M, 0, "plain_fp32"), dtype=torch.uint8, device="cuda")
    del ws
    steps = max(10, args.steps // 10)

    def timeit(fn):
        for i in range(3):
            fn(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            fn(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def plain(i):
        S, y, yb, sb = sets[i % len(sets)]
        T.transform_forward(S, taps, K, M, out=y, compute="plain_fp32")
        T.transform_adjoint(yb, taps, K, M, out=sb, compute="plain_fp32")

    t = timeit(plain)
    res["plain_fp32"] = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
                         "speedup_fused_over_plain": round(blocks_per_s / (B / t), 2)}

    def rocfft(i):
        S, y, yb, sb = sets[i % len(sets)]
        y.copy_(torch.fft.ifft(S * taps, dim=-1, norm="forward"))
        sb.copy_(taps * torch.fft.fft(yb, dim=-1))

    t = timeit(rocfft)
    res["torch_fft_rocfft"] = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
                               "speedup_fused_over_rocfft": round(blocks_per_s / (B / t), 2),
                               "note": "torch.mul + torch.fft (rocFFT) + copy, not fused"}
    return res


def cpu_baseline(S_h, taps_h, seconds):
    """The FP64 oracle (plain O(N^2) C, OpenMP over blocks) on a bounded sample of
    the same workload: forward + adjoint of the first blocks."""
    import numpy as np
    from oracle import oracle as O
    O.build()
    nth = O.max_threads()
    yb = np.ones_like(S_h[:1])
    t0 = time.perf_counter()
    O.forward(S_h[:nth], taps_h)
    O.adjoint(np.repeat(yb, nth, axis=0), taps_h)
    t1 = time.perf_counter() - t0
    per_round = max(t1, 1e-3)
    rounds = max(1, int(seconds / per_round))
    nb = min(S_h.shape[0], nth * rounds)
    t0 = time.perf_counter()
    y = O.forward(S_h[:nb], taps_h)
    O.adjoint(y, taps_h)
    dt = time.perf_counter() - t0
    return {"value": round(nb / dt, 2), "unit": "blocks/s", "cores": nth, "kind": "oracle",
            "sample": f"first {nb} of 4096 blocks (K=128, M=15), forward + adjoint, FP64 O(N^2), "
                      f"{dt:.1f} s on {nth} threads"}


if __name__ == "__main__":
    main()

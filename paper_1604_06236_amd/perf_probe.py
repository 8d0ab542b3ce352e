"""Run selected transforms a few times for profiling (rocprofv3 counters/traces).

    python -m paper_1604_06236_amd.perf_probe --what forward --reps 5

Also runs a device-to-device copy of a known size (--copy-mib), whose FETCH_SIZE
and WRITE_SIZE readings calibrate the counters: the copy reads and writes exactly
that many bytes.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--what", default="forward",
                    choices=["forward", "adjoint", "forward_adjoint", "ragged", "split_bf16",
                             "split_fp16", "differentiation", "decimated", "nufft", "schedules", "all"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--config", default=None,
                    help="workload for forward/adjoint/forward_adjoint (default: plain_gpu)")
    args = ap.parse_args()

    import numpy as np
    import torch
    from paper_1604_06236_amd import transform as T
    from paper_1604_06236_amd import workloads as W

    dev = "cuda"
    n = args.copy_mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(args.reps):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b

    if args.what == "all":
        for w in ("forward_adjoint", "ragged", "split_bf16", "split_fp16", "differentiation", "decimated"):
            run(w, args.reps, T, W, np, torch)
        return
    run(args.what, args.reps, T, W, np, torch, args.config)


def run(what, reps, T, W, np, torch, config=None):
    dev = "cuda"
    if what == "nufft":
        from paper_1604_06236_amd import nufft as NU
        B, P, eta = 256, 1024, 6
        a = NU.damping_for(1e-7, eta, P)
        rng = np.random.default_rng(11)
        t = torch.from_numpy(np.stack([W.jittered_instants(rng, P) for _ in range(B)])).to(dev)
        s = torch.from_numpy(W.cn01(rng, (B, P)).astype(np.complex64)).to(dev)
        S = torch.empty_like(s)
        for _ in range(reps):
            NU.nufft_type5(t, s, eta, a, out=S)
            NU.nufft_type5(t, s, eta, a, out=S, gridding=True)
        torch.cuda.synchronize()
        print(f"nufft: {reps} x type-5 solves (exact sums, then gridding) on {B} x P={P}, eta={eta}", flush=True)
        return
    if what == "decimated":
        c = W.CONFIGS["plain_gpu"]
        S_h, taps_h = W.make_uniform(c)
        S = torch.from_numpy(S_h).to(dev)
        taps = torch.from_numpy(taps_h).to(dev)
        d = torch.empty((c.nblocks, c.K), dtype=torch.complex64, device=dev)
        sb = torch.empty_like(S)
        for _ in range(reps):
            T.transform_decimated(S, taps, c.K, c.M, out=d)
            T.transform_decimated_adjoint(d, taps, c.K, c.M, out=sb)
        torch.cuda.synchronize()
        print(f"decimated: {reps} forward+adjoint on plain_gpu", flush=True)
        return
    if what == "ragged":
        lay, S_h, taps_h = W.make_ragged("ragged")
        plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total)
        S = torch.from_numpy(S_h).to(dev)
        taps = torch.from_numpy(taps_h).to(dev)
        y = torch.empty_like(S)
        sb = torch.empty_like(S)
        for _ in range(reps):
            plan.execute("forward", S, taps, out=y, use_graph=False)
            plan.execute("adjoint", y, taps, out=sb, use_graph=False)
            plan.execute("adjoint", y, taps, out=sb, aux=S, want_taps_bar=True, use_graph=False)
        torch.cuda.synchronize()
        plan.close()
        print(f"ragged: {reps} x (forward, adjoint, adjoint with tap gradient) over {lay.K.size} blocks",
              flush=True)
        return
    if what == "schedules":
        # Every fused schedule for the workload's (K, M), in table order, at grid cap 1024:
        # the dispatch sequence is (forward, adjoint) x reps per schedule.
        c = W.CONFIGS[config or "precision"]
        S_h, taps_h = W.make_uniform(c)
        S = torch.from_numpy(S_h).to(dev)
        taps = torch.from_numpy(taps_h).to(dev)
        y = torch.empty_like(S)
        sb = torch.empty_like(S)
        idx0, cap0, _ = T.selected_schedule(c.K, c.M)
        try:
            for idx, d in enumerate(T.schedules(c.K, c.M)):
                T.select_schedule(c.K, c.M, idx, grid_cap=1024)
                for _ in range(reps):
                    T.transform_forward(S, taps, c.K, c.M, out=y)
                    T.transform_adjoint(y, taps, c.K, c.M, out=sb)
                torch.cuda.synchronize()
                print(idx, d["radices"], d["threads_per_block"], d["nontemporal"], flush=True)
        finally:
            T.select_schedule(c.K, c.M, idx0, cap0)
        return
    cfg = {"split_bf16": "precision", "split_fp16": "precision",
           "differentiation": "differentiation"}.get(what, config or "plain_gpu")
    c = W.CONFIGS[cfg]
    S_h, taps_h = W.make_uniform(c)
    S = torch.from_numpy(S_h).to(dev)
    taps = torch.from_numpy(taps_h).to(dev)
    y = torch.empty_like(S)
    compute = what if what.startswith("split") else "fp32"
    for _ in range(reps):
        if what in ("forward", "forward_adjoint", "split_bf16", "split_fp16", "differentiation"):
            T.transform_forward(S, taps, c.K, c.M, out=y, compute=compute)
        if what in ("adjoint", "forward_adjoint"):
            T.transform_adjoint(S, taps, c.K, c.M, out=y)
        if what == "differentiation":
            T.transform_adjoint(y, taps, c.K, c.M, coeffs=S, want_taps_bar=True)
    torch.cuda.synchronize()
    print(f"{what}: {reps} reps on {cfg} ({c.nblocks} blocks, K={c.K}, M={c.M})", flush=True)


if __name__ == "__main__":
    main()

"""Schedule autotuner for the fused kernels.

For a block shape (K, M) the library compiles several schedules (radix plan,
threads per block, blocks per workgroup, prefetch, twiddle form).  The tuner
times forward + adjoint for each schedule and grid cap on synthetic batches of
the given size, selects the fastest in the library and can save the choices as
JSON ({"K,M": [schedule, grid_cap]}), which `transform` loads at import from
$BT_SCHEDULES or from schedules.json next to this file.

    python -m paper_1604_06236_amd.autotune --out schedules.json

The ragged kernel's work-item size and its per-class tile pipelining (prefetch on or off
per class and body) are tuned and saved alongside.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (K, M, blocks) of the standard workloads, plus the classes of ragged batches
STANDARD = [(16, 5, 65536), (128, 15, 4096), (256, 9, 8192), (1024, 15, 2048)]


def _time_pairs(torch, calls, reps, rounds=3):
    """Seconds per forward + adjoint pair: HIP events around `reps` back-to-back
    pairs rotating over the buffer sets; the minimum over `rounds` runs."""
    best = float("inf")
    for _ in range(rounds):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for i in range(reps):
            fwd, adj = calls[i % len(calls)]
            fwd()
            adj()
        ev1.record()
        torch.cuda.synchronize()
        best = min(best, ev0.elapsed_time(ev1) * 1e-3 / reps)
    return best


def tune_shape(T, K, M, B, caps=(0, 256, 512, 1024, 2048), reps=50, nbuf=4, verbose=True):
    """Time every compiled schedule of (K, M) at several grid caps on a batch of B
    blocks: forward S -> y and adjoint yb -> sb over `nbuf` rotating buffer sets
    (separate buffers, so neither direction reads what the other just touched)."""
    import torch
    N = K * M
    dev = "cuda"
    taps = torch.rand(N, device=dev) + 0.5
    sets = [tuple(torch.randn(B, N, dtype=torch.complex64, device=dev) for _ in range(4))
            for _ in range(nbuf)]
    results = []
    for idx, desc in enumerate(T.schedules(K, M)):
        for cap in caps:
            T.select_schedule(K, M, idx, cap)
            calls = [(T.bind_forward(S, taps, K, M, y), T.bind_adjoint(yb, taps, K, M, sb))
                     for (S, y, yb, sb) in sets]
            for i in range(2 * nbuf):
                calls[i % nbuf][0]()
                calls[i % nbuf][1]()
            torch.cuda.synchronize()
            t = _time_pairs(torch, calls, reps)
            results.append({"schedule": idx, "grid_cap": cap, "us_fwd_adj": round(t * 1e6, 2),
                            "GBps": round(2 * 16.0 * N * B / t / 1e9, 1), **desc})
            if verbose:
                print(f"K={K} M={M} sched={idx} cap={cap} {desc['radices']} TB={desc['threads_per_block']} "
                      f"BPW={desc['blocks_per_workgroup']} pf={desc['prefetch']} "
                      f"seq={desc['sequential_twiddles']} paired={desc['paired_io']} nt={desc['nontemporal']}: "
                      f"{t * 1e6:.1f} us", flush=True)
    best = min(results, key=lambda r: r["us_fwd_adj"])
    T.select_schedule(K, M, best["schedule"], best["grid_cap"])
    return best, results


def tune_ragged(T, W, chunks=(1, 2, 3, 4, 6, 8), reps=10, verbose=True):
    """Time forward + adjoint of the standard ragged batch for several work-item
    sizes (tiles per item); returns the best size."""
    import numpy as np
    import torch
    lay, S_h, taps_h = W.make_ragged("ragged")
    S = torch.from_numpy(S_h).cuda()
    taps = torch.from_numpy(taps_h).cuda()
    yb = torch.randn(lay.total, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(S)
    sb = torch.empty_like(S)
    results = []
    for c in chunks:
        plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total, chunk_tiles=c)
        for _ in range(2):
            plan.execute("forward", S, taps, out=y)
            plan.execute("adjoint", yb, taps, out=sb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.execute("forward", S, taps, out=y)
            plan.execute("adjoint", yb, taps, out=sb)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        plan.close()
        results.append({"chunk_tiles": c, "us_fwd_adj": round(t * 1e6, 1),
                        "GBps": round(2 * 20.0 * lay.total / t / 1e9, 1)})
        if verbose:
            print(f"ragged chunk_tiles={c}: {t * 1e6:.1f} us", flush=True)
    best = min(results, key=lambda r: r["us_fwd_adj"])
    return best, results


RAGGED_CLASSES = [(K, M) for K in (64, 128, 256, 512, 1024) for M in (3, 5, 7, 9, 15)]


def tune_ragged_prefetch(T, classes=RAGGED_CLASSES, reps=20, verbose=True):
    """For each class of the ragged kernel and each of its three bodies (0 forward, 1 output
    side, 2 adjoint with tap gradient) that has a prefetching form, time a single-class batch
    (per-block taps, about 250 MB per array) with the prefetch on and off and select the faster.
    Returns {"KxM": [choice per body]} (0 off, 1 on; keyed unlike the fused schedules'
    "K,M" entries, which the library's loader reads) and every timing."""
    import numpy as np
    import torch
    dev = "cuda"
    choice, report = {}, {}
    for K, M in classes:
        for b in range(3):
            T.ragged_prefetch_select(K, M, b, -1)
        on = [T.ragged_prefetch_selected(K, M, b) for b in range(3)]
        if not any(on):
            continue
        N = K * M
        B = int(250e6 // (N * 8))
        g = torch.Generator(device=dev).manual_seed(K * 64 + M)
        S = torch.randn(B * N, dtype=torch.complex64, device=dev, generator=g)
        taps = torch.rand(B * N, device=dev, generator=g) + 0.5
        y = S.clone()
        sb = torch.empty_like(S)
        tb = torch.empty(B * N, dtype=torch.float32, device=dev)
        off = np.arange(B, dtype=np.int64) * N
        sel = []
        for b in range(3):
            if not on[b]:
                sel.append(0)
                continue
            times = {}
            for pf in (1, 0):
                T.ragged_prefetch_select(K, M, b, pf)
                plan = T.RaggedPlan(np.full(B, K), np.full(B, M), off, off, B * N)
                if b == 0:
                    call = plan.bind("forward", S, taps, y)
                elif b == 1:
                    call = plan.bind("adjoint", y, taps, sb)
                else:
                    call = plan.bind("adjoint", y, taps, sb, aux=S, taps_bar=tb)
                best = float("inf")
                for _ in range(3):
                    for _ in range(2):
                        call()
                    ev0 = torch.cuda.Event(enable_timing=True)
                    ev1 = torch.cuda.Event(enable_timing=True)
                    ev0.record()
                    for _ in range(reps):
                        call()
                    ev1.record()
                    torch.cuda.synchronize()
                    best = min(best, ev0.elapsed_time(ev1) * 1e3 / reps)
                plan.close()
                times[pf] = best
            pick = 1 if times[1] <= times[0] else 0
            T.ragged_prefetch_select(K, M, b, pick)
            sel.append(pick)
            report[f"{K},{M},{b}"] = {"us_prefetch": round(times[1], 2), "us_no_prefetch": round(times[0], 2)}
            if verbose:
                print(f"ragged ({K}, {M}) body {b}: prefetch {times[1]:.1f} us, without {times[0]:.1f} us "
                      f"-> {'on' if pick else 'off'}", flush=True)
        choice[f"{K}x{M}"] = sel
        del S, taps, y, sb, tb
        torch.cuda.empty_cache()
    return choice, report


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="write the selections here (JSON)")
    ap.add_argument("--report", default=None, help="write every timing here (JSON)")
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--only-ragged-prefetch", action="store_true",
                    help="tune only the ragged kernel's per-class prefetch, keeping the other "
                         "selections of --out (or of the loaded schedules)")
    args = ap.parse_args()
    from paper_1604_06236_amd import transform as T
    from paper_1604_06236_amd import _native as nat
    if args.only_ragged_prefetch:
        choice, report = tune_ragged_prefetch(T)
        if args.out:
            src = args.out if os.path.exists(args.out) else os.path.join(
                os.path.dirname(os.path.abspath(__file__)), "schedules.json")
            with open(src) as f:
                sel = json.load(f)
            sel["ragged_prefetch"] = choice
            with open(args.out, "w") as f:
                json.dump(sel, f, indent=1)
        if args.report:
            with open(args.report, "w") as f:
                json.dump(report, f, indent=1)
        return
    report = {}
    for K, M, B in STANDARD:
        best, res = tune_shape(T, K, M, B, reps=args.reps)
        report[f"{K},{M}"] = {"best": best, "all": res}
        print(f"best for K={K} M={M}: schedule {best['schedule']} cap {best['grid_cap']} "
              f"({best['us_fwd_adj']} us, {best['GBps']} GB/s)", flush=True)
    from paper_1604_06236_amd import workloads as W
    best_r, res_r = tune_ragged(T, W)
    report["ragged"] = {"best": best_r, "all": res_r}
    pf_r, pf_rep = tune_ragged_prefetch(T)
    report["ragged_prefetch"] = pf_rep
    print(f"best for ragged: chunk_tiles {best_r['chunk_tiles']} ({best_r['us_fwd_adj']} us, "
          f"{best_r['GBps']} GB/s)", flush=True)
    if args.out:
        nat.check("transform_save_schedule", nat.load().transform_save_schedule(args.out.encode()))
        with open(args.out) as f:
            sel = json.load(f)
        sel["ragged_chunk_tiles"] = best_r["chunk_tiles"]
        sel["ragged_prefetch"] = pf_r
        with open(args.out, "w") as f:
            json.dump(sel, f, indent=1)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()

"""Benchmark of the block-transform library on one MI355X.

Headline step: one forward plus one adjoint transform of the ragged batch --
10,000 blocks whose K is drawn from {64, 128, 256, 512, 1024} and M from
{3, 5, 7, 9, 15}, seeded 64-QAM coefficients, one raised-cosine filter per
block with roll-off U[0.1, 0.9] -- each direction one launch (one workgroup
per cost-ordered work item) replayed from a HIP graph, inputs resident in HBM.  It is the largest of the
standard single-GPU batches (30.7 M points; 1.23 GB of algorithmic traffic
per step, far above the 256 MB last-level cache).

Prints one JSON line: blocks/s over forward + adjoint; the roofline of the
dominant kernel (the ragged forward) from HIP events recorded around its
launches on its stream; the unfused plain-FP32 path on the same blocks; the
error against the FP64 oracle; the other standard workloads with their own
rooflines and plain-FP32 speedups; and the oracle timed on the host cores
(one thread and all threads, median of five runs) over a bounded seeded
sample of the ragged batch.

`--profile-workload NAME` instead runs one workload's kernels a few times
(rotating buffer sets, after a 256 MiB device copy whose counter readings
calibrate FETCH_SIZE / WRITE_SIZE) for rocprofv3, prints what it ran, and
exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "blocks/s and % of HBM/MFMA peak, fwd+adjoint, vs plain FP32 at stated error"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK = 2.5e15
TOL = 1e-5
# sources each roofline's counter entry in profiles/traffic.json was taken on
KERNEL_SOURCES = {
    "ragged": ("bt_ragged.hip", "bt_half.hpp", "bt_fused.hpp", "bt_dft.hpp"),
    "fused": ("bt_fused.hpp", "bt_dft.hpp"),
    "fused_half": ("bt_fused_half.hip", "bt_half.hpp", "bt_fused.hpp", "bt_dft.hpp"),
}
PROFILE_WORKLOADS = ("ragged", "ragged_class", "plain_gpu", "precision", "split_bf16", "split_fp16",
                     "differentiation", "decimated", "nufft", "schedules", "copy")


def kernel_hash(kind: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1604_06236_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name: str, kind: str, schedule=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel sources (and the same schedule); null otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            e = json.load(f)[name]
        if e.get("kernel_hash") != kernel_hash(kind):
            return None
        if schedule is not None and e.get("schedule") != list(schedule):
            return None
        return float(e["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError, TypeError):
        return None


def _rel(a, b):
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _events_ms(calls, reps):
    """Average duration of one call, from HIP events recorded on the launch stream (the
    current torch stream, which every bound call launches on) around `reps` back-to-back
    calls rotating over `calls`."""
    import torch
    for c in calls:
        c()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(reps):
        calls[i % len(calls)]()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def _timeit(fn, steps, warmup=3, warm_s=0.2):
    """Seconds per call of fn(i) over `steps` calls, after `warmup` calls and an untimed
    pre-warm of about warm_s seconds (the GPU may have idled during host work, such as an
    oracle reference, and its clocks need to settle)."""
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < warm_s and i < 10000:
        fn(i)
        i += 1
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn(i)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _roofline(alg_bytes, ms, traffic, kernel, extra=None):
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
         "kernel_ms": round(ms, 5), "algorithmic_bytes_per_launch": alg_bytes}
    if extra:
        r.update(extra)
    return r


# ---------------------------------------------------------------------------- ragged batch
class RaggedBatch:
    """The ragged workload on the device: `nbuf` buffer sets (S, y, ybar, Sbar)."""

    def __init__(self, T, W, nbuf=2):
        import numpy as np
        import torch
        self.lay, self.S_h, self.taps_h = W.make_ragged("ragged")
        lay = self.lay
        self.nblocks = int(lay.K.size)
        self.points = lay.total
        r_y = W.rng_streams(W.CONFIGS["ragged"].seed + 100, 1)[0]
        self.yb_h = W.cn01(r_y, lay.total).astype(np.complex64)
        self.plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total)
        self.taps = torch.from_numpy(self.taps_h).cuda()
        self.sets = []
        rng = np.random.default_rng(1234)
        for i in range(nbuf):
            S = torch.from_numpy(self.S_h if i == 0 else W.qam(rng, 64, lay.total).astype(np.complex64)).cuda()
            yb = torch.from_numpy(self.yb_h if i == 0 else W.cn01(rng, lay.total).astype(np.complex64)).cuda()
            self.sets.append((S, torch.empty_like(S), yb, torch.empty_like(S)))
        self.fwd = [self.plan.bind("forward", S, self.taps, y) for (S, y, yb, sb) in self.sets]
        self.adj = [self.plan.bind("adjoint", yb, self.taps, sb) for (S, y, yb, sb) in self.sets]

    def close(self):
        self.plan.close()


def headline(args, T, W):
    import numpy as np
    import torch
    from oracle import fftref as F
    from oracle import oracle as O
    rb = RaggedBatch(T, W, args.nbuf)
    B = rb.nblocks

    def step(i):
        rb.fwd[i % len(rb.fwd)]()
        rb.adj[i % len(rb.adj)]()

    # untimed pre-warm (first launches capture the graphs; cold clocks run slower)
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < 0.3 and i < 2000:
        step(i)
        i += 1
        if i % 16 == 0:
            torch.cuda.synchronize()
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    blocks_per_s = B / (ms_per_step * 1e-3)

    fwd_ms = _events_ms(rb.fwd, args.steps)
    adj_ms = _events_ms(rb.adj, args.steps)
    # algorithmic bytes of one ragged forward: read S (8 B) and the block's own tap (4 B),
    # write y (8 B), per point
    alg = 20.0 * rb.points
    roof = _roofline(alg, fwd_ms, measured_traffic("ragged_forward_10000", "ragged"),
                     "ragged_kernel (forward), one launch per direction from a HIP graph",
                     {"adjoint_kernel_ms": round(adj_ms, 5),
                      "timing": f"HIP events around {args.steps} back-to-back graph launches per direction"})

    # error of the timed data against the oracle: every block against the FFT form of the
    # oracle, 40 seeded blocks against the O(N^2) sums
    S0, y0, yb0, sb0 = rb.sets[0]
    rb.fwd[0]()
    rb.adj[0]()
    torch.cuda.synchronize()
    yh, sbh = y0.cpu().numpy(), sb0.cpu().numpy()
    lay = rb.lay
    args3 = (lay.N, lay.x_off, lay.tap_off)
    y_ref = F.forward_ragged(*args3, rb.S_h, rb.taps_h)
    sb_ref, _ = F.adjoint_ragged(*args3, rb.yb_h, rb.taps_h)
    idx = np.sort(np.random.default_rng(1).choice(B, 40, replace=False))
    sub = lay.subset(idx)

    def pick(x):
        return np.concatenate([x[int(lay.x_off[b]):int(lay.x_off[b] + lay.N[b])] for b in idx])
    sargs = (sub.N, sub.x_off, sub.tap_off)
    error = {"rel_l2_forward": _rel(yh, y_ref), "rel_l2_adjoint": _rel(sbh, sb_ref),
             "rel_l2_forward_sums_sample": _rel(pick(yh), O.forward_ragged(*sargs, pick(rb.S_h), pick(rb.taps_h))),
             "tolerance": TOL, "blocks_checked": B,
             "reference": "FP64 oracle: FFT form on every block, O(N^2) sums on 40 seeded blocks"}
    del y_ref, sb_ref

    out = {"metric": METRIC, "value": round(blocks_per_s, 1), "unit": "blocks/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded 64-QAM coefficients, per-block raised-cosine filters, roll-off U[0.1, 0.9])",
           "config": {"workload": "ragged: 10000 blocks, K in {64,128,256,512,1024}, M in {3,5,7,9,15} "
                                  "(30.7 M points), per-block taps; forward + adjoint, one launch "
                                  "each from a HIP graph",
                      "blocks": B, "points": rb.points, "taps": "per block", "buffer_sets": args.nbuf},
           "roofline": roof, "error": error}
    if not args.no_compare:
        out["compare"] = {"plain_fp32": ragged_plain(T, rb, blocks_per_s, args)}
    rb.close()
    return out


def ragged_plain(T, rb, blocks_per_s, args):
    """The ragged batch through the unfused plain-FP32 path: the blocks of each (K, M) class
    gathered into a uniform batch, forward + adjoint per class, summed over the classes."""
    import numpy as np
    import torch
    lay = rb.lay
    calls = []
    keep = []
    for K, M in sorted(set(zip(lay.K.tolist(), lay.M.tolist()))):
        idx = np.nonzero((lay.K == K) & (lay.M == M))[0]
        N = K * M
        take = lambda x, off: np.stack([x[int(off[b]):int(off[b] + N)] for b in idx])
        S = torch.from_numpy(take(rb.S_h, lay.x_off)).cuda()
        tp = torch.from_numpy(take(rb.taps_h, lay.tap_off)).cuda()
        yb = torch.from_numpy(take(rb.yb_h, lay.x_off)).cuda()
        y, sb = torch.empty_like(S), torch.empty_like(S)
        T.transform_prepare(K, M, "plain_fp32")
        calls.append(T.bind_forward(S, tp, K, M, y, compute="plain_fp32"))
        calls.append(T.bind_adjoint(yb, tp, K, M, sb, compute="plain_fp32"))
        keep.append((S, tp, yb, y, sb))

    def pstep(i):
        for c in calls:
            c()

    t = _timeit(pstep, max(5, args.steps // 10))
    return {"blocks_per_s": round(rb.nblocks / t, 1), "ms_per_step": round(t * 1e3, 4),
            "speedup_over_plain": round(blocks_per_s / (rb.nblocks / t), 2),
            "note": "unfused plain FP32: one launch per stage, the 25 (K, M) classes as 25 uniform batches"}


# ---------------------------------------------------------------------------- uniform workloads
def _uniform_sets(W, cfg, nbuf, seed):
    import numpy as np
    import torch
    c = W.CONFIGS[cfg]
    S_h, taps_h = W.make_uniform(cfg)
    B, N = S_h.shape
    rng = np.random.default_rng(seed)
    yb_h = W.cn01(W.rng_streams(c.seed + 100, 1)[0], (B, N)).astype(np.complex64)
    sets = []
    for i in range(nbuf):
        S = torch.from_numpy(S_h if i == 0 else W.cn01(rng, (B, N)).astype(np.complex64)).cuda()
        yb = torch.from_numpy(yb_h if i == 0 else W.cn01(rng, (B, N)).astype(np.complex64)).cuda()
        sets.append((S, torch.empty_like(S), yb, torch.empty_like(S)))
    return c, S_h, taps_h, yb_h, torch.from_numpy(taps_h).cuda(), sets


def uniform_workload(T, W, cfg, args, nbuf, tapgrad=False, rocfft=False, roof_name=None):
    """Forward + adjoint (with the shared tap gradient if `tapgrad`) over `nbuf` rotating
    buffer sets: blocks/s, the forward kernel's roofline, the error against the oracle and
    the plain-FP32 path on the same data."""
    import numpy as np
    import torch
    from oracle import oracle as O
    c, S_h, taps_h, yb_h, taps, sets = _uniform_sets(W, cfg, nbuf, seed=W.CONFIGS[cfg].seed + 1000)
    K, M = c.K, c.M
    B, N = S_h.shape
    tb = torch.empty(N, dtype=torch.float32, device="cuda") if tapgrad else None
    T.transform_prepare(K, M)
    fwd = [T.bind_forward(S, taps, K, M, y) for (S, y, yb, sb) in sets]
    adj = [T.bind_adjoint(yb, taps, K, M, sb, coeffs=S if tapgrad else None, taps_bar=tb)
           for (S, y, yb, sb) in sets]

    def step(i):
        fwd[i % nbuf]()
        adj[i % nbuf]()

    steps = max(20, args.steps // 2)
    t = _timeit(step, steps)
    fwd_ms = _events_ms(fwd, steps)
    adj_ms = _events_ms(adj, steps)
    # algorithmic bytes: forward reads S and writes y (16 B per point) plus the shared taps
    # once; the adjoint the same, plus S (8 B per point) when it forms the tap gradient
    fwd_bytes = 16.0 * B * N + 4.0 * N
    step_bytes = 2 * fwd_bytes + (8.0 * B * N if tapgrad else 0.0)
    sched = T.selected_schedule(K, M)
    half = bool(sched[2].get("half_lds"))
    kind = "fused_half" if half else "fused"
    res = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
           "achieved_GBps": round(step_bytes / t / 1e9, 1),
           "frac_hbm_peak": round(step_bytes / t / 1e9 / HBM_PEAK_GBS, 4),
           "roofline": _roofline(fwd_bytes, fwd_ms,
                                 measured_traffic(roof_name, kind, sched[:2]) if roof_name else None,
                                 "%s (forward), schedule %s" % ("half_lds_kernel" if half else "fused_kernel",
                                                                json.dumps(sched[2])),
                                 {"adjoint_kernel_ms": round(adj_ms, 5)})}
    # error of the timed data on a seeded sample against the O(N^2) sums
    S0, y0, yb0, sb0 = sets[0]
    step(0)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(0).choice(B, min(B, 32), replace=False))
    res["error"] = {"rel_l2_forward": _rel(y0.cpu().numpy()[idx], O.forward(S_h[idx], taps_h)),
                    "rel_l2_adjoint": _rel(sb0.cpu().numpy()[idx], O.adjoint(yb_h[idx], taps_h)[0]),
                    "blocks_checked": int(idx.size), "tolerance": TOL}
    if not args.no_compare:
        T.transform_prepare(K, M, "plain_fp32")
        pf = [T.bind_forward(S, taps, K, M, y, compute="plain_fp32") for (S, y, yb, sb) in sets]
        pa = [T.bind_adjoint(yb, taps, K, M, sb, coeffs=S if tapgrad else None, taps_bar=tb,
                             compute="plain_fp32") for (S, y, yb, sb) in sets]

        def pstep(i):
            pf[i % nbuf]()
            pa[i % nbuf]()

        tp = _timeit(pstep, max(5, steps // 5))
        res["plain_fp32"] = {"blocks_per_s": round(B / tp, 1), "ms_per_step": round(tp * 1e3, 4),
                             "speedup_over_plain": round(tp / t, 2)}
        del pf, pa
        if rocfft:
            def rstep(i):
                S, y, yb, sb = sets[i % nbuf]
                y.copy_(torch.fft.ifft(S * taps, dim=-1, norm="forward"))
                sb.copy_(taps * torch.fft.fft(yb, dim=-1))
            tr = _timeit(rstep, max(5, steps // 5))
            res["torch_fft_rocfft"] = {"blocks_per_s": round(B / tr, 1), "ms_per_step": round(tr * 1e3, 4),
                                       "speedup_over_rocfft": round(tr / t, 2),
                                       "note": "torch.mul + torch.fft (rocFFT) + copy, not fused"}
    return res, sets, taps


def precision_workload(T, W, args):
    """K = 1024, M = 15: the FFT path and the split-precision MFMA paths, forward + adjoint."""
    import numpy as np
    import torch
    from oracle import oracle as O
    res, sets, taps = uniform_workload(T, W, "precision", args, nbuf=2, roof_name="fused_forward_1024x15")
    c = W.CONFIGS["precision"]
    K, M, B = c.K, c.M, c.nblocks
    N = K * M
    S_h, taps_h = W.make_uniform("precision")
    idx = np.array([0, 777, 2047])
    ref = O.forward(S_h[idx], taps_h)
    out = {"fp32": res}
    # executed MFMA flops per block and direction: stage A 64 tiles x 12 (16x16x16),
    # stages B 15 rows x 96 (16x16x32)
    mfma_flops = (64 * 12 * 16 * 16 * 16 * 2 + M * 96 * 16 * 16 * 32 * 2) * B
    for compute in ("split_bf16", "split_fp16"):
        pf = [T.bind_forward(S, taps, K, M, y, compute=compute) for (S, y, yb, sb) in sets]
        pa = [T.bind_adjoint(yb, taps, K, M, sb, compute=compute) for (S, y, yb, sb) in sets]

        def pstep(i, pf=pf, pa=pa):
            pf[i % len(pf)]()
            pa[i % len(pa)]()

        t = _timeit(pstep, max(10, args.steps // 5))
        fms = _events_ms(pf, 20)
        pf[0]()
        torch.cuda.synchronize()
        err_y = sets[0][1].cpu().numpy()[idx]
        byts = 2 * 16.0 * N * B
        out[compute] = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
                        "achieved_GBps": round(byts / t / 1e9, 1),
                        "frac_hbm_peak": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
                        "forward_kernel_ms": round(fms, 5),
                        "rel_l2_forward": _rel(err_y, ref), "max_abs_forward": float(np.abs(err_y - ref).max()),
                        "mfma_TFLOPs_executed": round(2 * mfma_flops / t / 1e12, 2),
                        "mfma_utilisation": round(2 * mfma_flops / t / MFMA_BF16_PEAK, 4),
                        "speedup_over_plain": round(res["plain_fp32"]["ms_per_step"] / (t * 1e3), 2)
                        if "plain_fp32" in res else None}
    del sets
    return out


def extras(T, W, args):
    """The other standard workloads, each forward + adjoint on one full batch."""
    import numpy as np
    import torch
    from oracle import oracle as O
    res = {}
    dev = "cuda"

    # ---- the 4096 x (128, 15) batch with the shared root-raised-cosine filter
    r, sets, _ = uniform_workload(T, W, "plain_gpu", args, nbuf=4, rocfft=True, roof_name="fused_forward_128x15")
    r["workload"] = "4096 blocks, K=128, M=15, shared RRC taps; forward + adjoint, four rotating buffer sets"
    res["plain_gpu"] = r
    del sets
    torch.cuda.empty_cache()

    # ---- precision workload: K=1024, M=15, 2048 blocks; FFT path and split MFMA paths
    res["precision"] = precision_workload(T, W, args)
    torch.cuda.empty_cache()

    # ---- differentiation workload: forward + adjoint with the shared tap gradient
    r, sets, _ = uniform_workload(T, W, "differentiation", args, nbuf=2, tapgrad=True,
                                  roof_name="fused_forward_256x9")
    r["workload"] = ("8192 blocks K=256 M=9, forward + adjoint with the deterministic shared "
                     "tap-gradient reduction, two rotating buffer sets")
    res["differentiation"] = r
    del sets
    torch.cuda.empty_cache()

    # ---- decimated eq. (7) operator on the 4096 x (128, 15) shape
    cfg = W.CONFIGS["plain_gpu"]
    K, M, B = cfg.K, cfg.M, cfg.nblocks
    N = K * M
    S_h, taps_h = W.make_uniform(cfg)
    S = torch.from_numpy(S_h).to(dev)
    taps = torch.from_numpy(taps_h).to(dev)
    d = torch.empty((B, K), dtype=torch.complex64, device=dev)
    db = torch.from_numpy(W.cn01(np.random.default_rng(10), (B, K)).astype(np.complex64)).to(dev)
    dsets = [(S, torch.empty_like(S))] + [(S.clone(), torch.empty_like(S)) for _ in range(3)]

    def decstep(i):
        Si, sbi = dsets[i % len(dsets)]
        T.transform_decimated(Si, taps, K, M, out=d)
        T.transform_decimated_adjoint(db, taps, K, M, out=sbi)

    t = _timeit(decstep, max(10, args.steps // 5))
    byts = (16.0 * N + 16.0 * K) * B
    idx = np.array([0, 2048, 4095])
    T.transform_decimated(S, taps, K, M, out=d)
    res["decimated"] = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
                        "achieved_GBps": round(byts / t / 1e9, 1),
                        "frac_hbm_peak": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
                        "rel_l2_forward": _rel(d.cpu().numpy()[idx], O.decimated(S_h[idx], taps_h, K)),
                        "workload": "eq. (7) on 4096 blocks K=128 M=15: forward (N -> K) + adjoint (K -> N)"}
    del S, taps, d, db, dsets
    torch.cuda.empty_cache()

    res["nufft"] = nufft_workload(args, W)
    return res


def nufft_workload(args, W):
    """Non-iterative type-5 / type-4 methods: 256 problems of P = 1024 jittered instants,
    eta = 6, truncation ratio mu = 1e-7 (eq. (49))."""
    import numpy as np
    import torch
    from oracle import lagrange as LG
    from paper_1604_06236_amd import nufft as NU
    dev = "cuda"
    steps = max(3, args.steps // 20)
    B, P, eta, mu = 256, 1024, 6, 1e-7
    a = NU.damping_for(mu, eta, P)
    rng = np.random.default_rng(11)
    t_h = np.stack([W.jittered_instants(rng, P) for _ in range(B)])
    s_h = W.cn01(rng, (B, P)).astype(np.complex64)
    A_h = W.cn01(rng, (B, P)).astype(np.complex64)
    tt = torch.from_numpy(t_h).to(dev)
    s = torch.from_numpy(s_h).to(dev)
    A = torch.from_numpy(A_h).to(dev)
    S5 = torch.empty_like(s)
    a4 = torch.empty_like(A)
    st = LG.Setup(t_h[0], eta, a)
    S_ref = LG.type5_method(t_h[0], s_h[0], eta, a, st)
    a_ref = LG.type4_method(t_h[0], A_h[0], eta, a, st)
    S_ge = LG.ge_type5(t_h[0], s_h[0])
    nres = {"workload": f"{B} problems of P={P} jittered instants (p/P + U[0, 0.6/P]), eta={eta}, "
                        f"mu={mu:g} (a={a:.4g}); one type-5 and one type-4 solve each per step",
            "oracle_method_vs_gaussian_elimination": _rel(S_ref, S_ge)}
    for name, refine, gridding in (("exact_sums", False, False), ("gridding", False, True),
                                   ("exact_sums_refined", True, False)):
        flags = (NU.NUFFT_REFINE if refine else 0) | (NU.NUFFT_GRIDDING if gridding else 0)
        ws = torch.empty(NU.nufft_workspace_size(B, P, eta, flags), dtype=torch.uint8, device=dev)

        def nstep(i, refine=refine, gridding=gridding, ws=ws):
            NU.nufft_type5(tt, s, eta, a, out=S5, workspace=ws, refine=refine, gridding=gridding)
            NU.nufft_type4(tt, A, eta, a, out=a4, workspace=ws, refine=refine, gridding=gridding)

        t = _timeit(nstep, steps)
        e = {"solves_per_s": round(2 * B / t, 1), "ms_per_step": round(t * 1e3, 4)}
        r5 = (LG.type5_refined(t_h[0], s_h[0], eta, a, st) if refine else S_ref)
        r4 = (LG.type4_refined(t_h[0], A_h[0], eta, a, st) if refine else a_ref)
        e["rel_l2_type5_vs_oracle"] = _rel(S5.cpu().numpy()[0], r5)
        e["rel_l2_type4_vs_oracle"] = _rel(a4.cpu().numpy()[0], r4)
        e["rel_l2_type5_vs_gaussian_elimination"] = _rel(S5.cpu().numpy()[0], S_ge)
        nres[name] = e
        del ws
    # the dominant kernel of the exact path: the type-1 sum of eq. (28) (unit amplitudes,
    # R = eta P outputs), timed alone with HIP events on the launch stream.  Executed work:
    # three real FP64 MFMA products per complex term (2 flops each)
    R = eta * P
    zt = torch.empty((B, R), dtype=torch.complex64, device=dev)
    NU.nudft_type1(tt, None, R, out=zt)
    reps = 20
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        NU.nudft_type1(tt, None, R, out=zt)
    ev1.record()
    torch.cuda.synchronize()
    t1 = ev0.elapsed_time(ev1) / reps * 1e-3
    tflops = 6.0 * B * P * R / t1 / 1e12
    nres["exact_type1_sum"] = {
        "shape": f"{B} problems, Q={P} instants -> R={R} outputs (eq. (28))",
        "us": round(t1 * 1e6, 1), "terms_per_s": float(f"{B * P * R / t1:.4g}"),
        "rel_l2_vs_oracle": _rel(zt[0].cpu().numpy(), LG.type1(t_h[0], np.ones(P), R)),
        "roofline": {"bound": "mfma", "dtype": "f64", "achieved": round(tflops, 2), "peak": 78.6,
                     "unit": "TFLOP/s", "frac": round(tflops / 78.6, 4),
                     "note": "executed FP64 MFMA work"}}
    return nres


# ---------------------------------------------------------------------------- CPU baseline
def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, runs=5):
    """The FP64 oracle (plain O(N^2) C, OpenMP over blocks) on a bounded seeded sample of
    the ragged batch, forward + adjoint: all host threads on 256 blocks and one thread on
    16 blocks, each the median of `runs` runs (blocks/s of the batch's own mix of sizes)."""
    import numpy as np
    from oracle import oracle as O
    O.build()
    nth = O.max_threads()
    lay, S_h, taps_h = W.make_ragged("ragged")
    rng = np.random.default_rng(2024)

    def sample(n):
        idx = np.sort(rng.choice(lay.K.size, n, replace=False))
        sub = lay.subset(idx)
        cat = lambda x, off: np.concatenate([x[int(off[b]):int(off[b] + lay.N[b])] for b in idx])
        return sub, cat(S_h, lay.x_off), cat(taps_h, lay.tap_off)

    def rate(sub, S, taps, threads):
        args = (sub.N, sub.x_off, sub.tap_off)
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            y = O.forward_ragged(*args, S, taps, nthreads=threads)
            O.adjoint_ragged(*args, y, taps, nthreads=threads)
            times.append(time.perf_counter() - t0)
        return sub.K.size / statistics.median(times), sum(times)

    all_rate, all_s = rate(*sample(256), nth)
    one_rate, one_s = rate(*sample(16), 1)
    return {"value": round(all_rate, 2), "unit": "blocks/s", "cores": nth, "kind": "oracle",
            "single_core_value": round(one_rate, 2), "cpu_model": cpu_model(), "runs": runs,
            "statistic": "median",
            "sample": f"seeded samples of the ragged batch, forward + adjoint, FP64 O(N^2) sums: "
                      f"256 blocks on {nth} threads ({all_s:.1f} s for {runs} runs) and 16 blocks on "
                      f"one thread ({one_s:.1f} s for {runs} runs); blocks/s of the batch's mix of "
                      f"sizes, extrapolated from the samples"}


# ---------------------------------------------------------------------------- profiling mode
def profile_workload(name, reps, T, W):
    """Run one workload's kernels `reps` times for rocprofv3 (rotating buffer sets), after a
    256 MiB device copy that calibrates the HBM counters."""
    import numpy as np
    import torch
    dev = "cuda"
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    if name == "copy":
        print("copy: 3 x 256 MiB device copy", flush=True)
        return
    if name == "ragged":
        rb = RaggedBatch(T, W, nbuf=2)
        tb = torch.empty(rb.points, dtype=torch.float32, device=dev)
        tg = [rb.plan.bind("adjoint", yb, rb.taps, sb, aux=S, taps_bar=tb) for (S, y, yb, sb) in rb.sets]
        for i in range(reps):
            rb.fwd[i % 2]()
            rb.adj[i % 2]()
            tg[i % 2]()
        torch.cuda.synchronize()
        rb.close()
        print(f"ragged: {reps} x (forward, adjoint, adjoint with tap gradient), 10000 blocks, graph replay",
              flush=True)
        return
    if name == "ragged_class":
        # one (K, M) class of the ragged batch (BT_CLASS="KxM", default 128x15), about 250 MB
        # per array with per-block taps: the ragged kernel (`reps` launches of the forward,
        # the adjoint and the adjoint with tap gradient) and then `reps` launches of the
        # uniform fused forward on the same data
        K, M = (int(v) for v in os.environ.get("BT_CLASS", "128x15").split("x"))
        N = K * M
        B = int(250e6 // (N * 8))
        rng = np.random.default_rng(8)
        S = torch.from_numpy(W.cn01(rng, (B, N)).astype(np.complex64)).to(dev)
        taps = torch.from_numpy(rng.uniform(0.5, 1.5, (B, N)).astype(np.float32)).to(dev)
        y = torch.empty_like(S)
        off = np.arange(B, dtype=np.int64) * N
        plan = T.RaggedPlan(np.full(B, K), np.full(B, M), off, off, B * N)
        fr = plan.bind("forward", S.view(-1), taps.view(-1), y.view(-1))
        sb = torch.empty_like(S)
        tb = torch.empty(B * N, dtype=torch.float32, device=dev)
        ar = plan.bind("adjoint", y.view(-1), taps.view(-1), sb.view(-1))
        gr = plan.bind("adjoint", y.view(-1), taps.view(-1), sb.view(-1), aux=S.view(-1), taps_bar=tb)
        for f in (fr, ar, gr):
            for _ in range(reps):
                f()
        torch.cuda.synchronize()
        ff = T.bind_forward(S, taps, K, M, y)
        for _ in range(reps):
            ff()
        torch.cuda.synchronize()
        plan.close()
        print(f"ragged_class: {reps} x ragged forward, adjoint, tap-gradient adjoint, then {reps} x fused "
              f"forward, {B} blocks of ({K}, {M})",
              flush=True)
        return
    if name == "nufft":
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
    if name == "decimated":
        c = W.CONFIGS["plain_gpu"]
        _, S_h, taps_h, _, taps, sets = _uniform_sets(W, "plain_gpu", 4, seed=5)
        d = torch.empty((c.nblocks, c.K), dtype=torch.complex64, device=dev)
        for i in range(reps):
            S, y, yb, sb = sets[i % 4]
            T.transform_decimated(S, taps, c.K, c.M, out=d)
            T.transform_decimated_adjoint(d, taps, c.K, c.M, out=sb)
        torch.cuda.synchronize()
        print(f"decimated: {reps} x (forward, adjoint) on 4096 x (128, 15), four buffer sets", flush=True)
        return
    if name == "schedules":
        # every fused schedule of the K=1024, M=15 batch, in table order, grid cap 1024:
        # (forward, adjoint) x reps per schedule
        c = W.CONFIGS["precision"]
        _, S_h, taps_h, _, taps, sets = _uniform_sets(W, "precision", 2, seed=6)
        idx0, cap0, _ = T.selected_schedule(c.K, c.M)
        try:
            for idx, d in enumerate(T.schedules(c.K, c.M)):
                T.select_schedule(c.K, c.M, idx, grid_cap=1024)
                for i in range(reps):
                    S, y, yb, sb = sets[i % 2]
                    T.transform_forward(S, taps, c.K, c.M, out=y)
                    T.transform_adjoint(yb, taps, c.K, c.M, out=sb)
                torch.cuda.synchronize()
                print(idx, d["radices"], d["threads_per_block"], d["nontemporal"], flush=True)
        finally:
            T.select_schedule(c.K, c.M, idx0, cap0)
        return
    cfg = {"split_bf16": "precision", "split_fp16": "precision"}.get(name, name)
    c = W.CONFIGS[cfg]
    nbuf = 4 if cfg == "plain_gpu" else 2
    _, S_h, taps_h, _, taps, sets = _uniform_sets(W, cfg, nbuf, seed=7)
    compute = name if name.startswith("split") else "fp32"
    tb = torch.empty(c.K * c.M, dtype=torch.float32, device=dev)
    for i in range(reps):
        S, y, yb, sb = sets[i % nbuf]
        T.transform_forward(S, taps, c.K, c.M, out=y, compute=compute)
        if name == "differentiation":
            T.transform_adjoint(yb, taps, c.K, c.M, out=sb, coeffs=S, taps_bar=tb)
        elif not name.startswith("split"):
            T.transform_adjoint(yb, taps, c.K, c.M, out=sb)
    torch.cuda.synchronize()
    what = "forward" if name.startswith("split") else "forward + adjoint"
    print(f"{name}: {reps} x {what} on {cfg} ({c.nblocks} blocks, K={c.K}, M={c.M}), {nbuf} buffer sets",
          flush=True)


# ---------------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nbuf", type=int, default=2, help="rotating buffer sets of the ragged batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain-FP32 / rocFFT comparison runs")
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads")
    ap.add_argument("--profile-workload", choices=PROFILE_WORKLOADS, default=None,
                    help="run one workload's kernels for a profiler and exit")
    ap.add_argument("--reps", type=int, default=5, help="repetitions in --profile-workload mode")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: every GPU box of this setup has "
                                   "one GPU, and the block transform has no cross-GPU step (blocks shard "
                                   "by index with no exchange)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1604_06236_amd import transform as T
    from paper_1604_06236_amd import workloads as W
    torch.cuda.set_device(0)

    if args.profile_workload:
        profile_workload(args.profile_workload, args.reps, T, W)
        return

    out = headline(args, T, W)
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["extras"] = extras(T, W, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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


def measured_traffic(name: str, schedule):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and the same schedule (null otherwise)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        e = d[name]
        if e.get("kernel_hash") != kernel_hash() or e.get("schedule") != list(schedule):
            return None
        return float(e["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError, TypeError):
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
    ap.add_argument("--no-extras", action="store_true", help="skip the other workloads")
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

    # pre-marshalled calls: the timed loop measures the GPU, not argument checking
    calls = [(T.bind_forward(S, taps, K, M, y), T.bind_adjoint(yb, taps, K, M, sb))
             for (S, y, yb, sb) in sets]

    def step(i):
        fwd, adj = calls[i % len(calls)]
        fwd()
        adj()

    # untimed pre-warm of about 0.3 s so the clocks have settled before the warmup steps
    # and the timed region (a 20-step warmup alone is about 1 ms; timed from a cold start
    # the first few hundred steps run about 10 % slower)
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < 0.3 and i < 20000:
        step(i)
        i += 1
        if i % 64 == 0:
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

    # kernel durations: HIP events (on the launch stream) around runs of back-to-back
    # launches of one kernel, rotating over the buffer sets
    def kernel_ms(which, reps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        for i in range(len(calls)):
            calls[i][which]()
        ev0.record()
        for i in range(reps):
            calls[i % len(calls)][which]()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    fwd_ms = kernel_ms(0, args.steps)
    adj_ms = kernel_ms(1, args.steps)
    step(0)

    # roofline of the forward kernel: algorithmic bytes = read S (8N) + write y (8N) per
    # block, plus the shared taps (4N) once per launch
    fwd_bytes = B * 16.0 * N + 4.0 * N
    achieved = fwd_bytes / (fwd_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("fused_forward_128x15", T.selected_schedule(K, M)[:2]),
                "kernel": "fused_kernel (forward), schedule %s" % json.dumps(T.selected_schedule(K, M)[2]),
                "kernel_ms": round(fwd_ms, 5), "adjoint_kernel_ms": round(adj_ms, 5),
                "algorithmic_bytes_per_launch": fwd_bytes,
                "timing": "HIP events around %d back-to-back launches per kernel" % args.steps}

    # error against the oracle on a seeded sample of blocks of the timed data
    from oracle import oracle as O
    S0, y0, yb0, sb0 = sets[0]
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

    if not args.no_extras:
        del sets, calls
        torch.cuda.empty_cache()
        out["extras"] = extras(T, W, args)

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
        return _timeit(fn, steps)

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


def _timeit(fn, steps, warmup=3, warm_s=0.2):
    """Seconds per call of fn over `steps` calls, after `warmup` calls and an untimed
    pre-warm of about warm_s seconds (the GPU may have idled during host work, such as
    an oracle reference, and its clocks need to settle)."""
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
    t0 = time.perf_counter()
    for i in range(steps):
        fn(i)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _rel(a, b):
    import numpy as np
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def extras(T, W, args):
    """The other standard workloads, each forward + adjoint on one full batch."""
    import numpy as np
    import torch
    from oracle import oracle as O
    res = {}
    steps = max(10, args.steps // 5)
    dev = "cuda"

    # ---- ragged batch: 10,000 blocks of mixed (K, M), per-block filters, one
    #      persistent launch per direction replayed from a HIP graph
    lay, S_h, taps_h = W.make_ragged("ragged")
    plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total)
    S = torch.from_numpy(S_h).to(dev)
    taps = torch.from_numpy(taps_h).to(dev)
    yb = torch.from_numpy(W.cn01(np.random.default_rng(7), lay.total).astype(np.complex64)).to(dev)
    y = torch.empty_like(S)
    sb = torch.empty_like(S)

    def rstep(i):
        plan.execute("forward", S, taps, out=y)
        plan.execute("adjoint", yb, taps, out=sb)

    t = _timeit(rstep, steps)
    nb = lay.K.size
    byts = 2 * 20.0 * lay.total            # per direction: read 8N + taps 4N, write 8N
    idx = np.array([0, 1234, 5678, nb - 1])
    yh = y.cpu().numpy()
    sub = lay.subset(idx)
    cat = lambda a, o, n: np.concatenate([a[int(o[b]):int(o[b] + n[b])] for b in idx])
    ref = O.forward_ragged(sub.N, sub.x_off, sub.tap_off, cat(S_h, lay.x_off, lay.N),
                           cat(taps_h, lay.tap_off, lay.N))
    res["ragged"] = {"blocks_per_s": round(nb / t, 1), "ms_per_step": round(t * 1e3, 4),
                     "achieved_GBps": round(byts / t / 1e9, 1),
                     "frac_hbm_peak": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
                     "rel_l2_forward_sampled": _rel(cat(yh, lay.x_off, lay.N), ref),
                     "workload": "10000 blocks, K in {64..1024}, M in {3,5,7,9,15}, per-block RC taps; "
                                 "forward + adjoint, one persistent launch each, HIP graph replay"}
    plan.close()
    del S, taps, yb, y, sb

    # ---- precision workload: K=1024, M=15, 2048 blocks; FFT path and split MFMA paths
    cfg = W.CONFIGS["precision"]
    K, M, B = cfg.K, cfg.M, cfg.nblocks
    N = K * M
    S_h, taps_h = W.make_uniform(cfg)
    S = torch.from_numpy(S_h).to(dev)
    taps = torch.from_numpy(taps_h).to(dev)
    yb = torch.from_numpy(W.cn01(np.random.default_rng(8), (B, N)).astype(np.complex64)).to(dev)
    y = torch.empty_like(S)
    sb = torch.empty_like(S)
    idx = np.array([0, 777, 2047])
    ref = O.forward(S_h[idx], taps_h)
    prec = {}
    # executed MFMA flops per block and direction: stage A 64 tiles x 12 (16x16x16),
    # stages B 15 rows x 96 (16x16x32)
    mfma_flops = (64 * 12 * 16 * 16 * 16 * 2 + M * 96 * 16 * 16 * 32 * 2) * B
    for compute in ("fp32", "split_bf16", "split_fp16"):
        pf = T.bind_forward(S, taps, K, M, y, compute=compute)
        pa = T.bind_adjoint(yb, taps, K, M, sb, compute=compute)

        def pstep(i, pf=pf, pa=pa):
            pf()
            pa()

        t = _timeit(pstep, steps)
        T.transform_forward(S, taps, K, M, out=y, compute=compute)
        err_y = y.cpu().numpy()[idx]
        byts = 2 * 16.0 * N * B
        e = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
             "achieved_GBps": round(byts / t / 1e9, 1),
             "frac_hbm_peak": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
             "rel_l2_forward": _rel(err_y, ref), "max_abs_forward": float(np.abs(err_y - ref).max())}
        if compute != "fp32":
            e["mfma_TFLOPs_executed"] = round(2 * mfma_flops / t / 1e12, 2)
            e["mfma_utilisation"] = round(2 * mfma_flops / t / 2.5e15, 4)
        prec[compute] = e
    res["precision"] = prec
    del S, taps, yb, y, sb

    # ---- decimated eq. (7) operator on the standard GPU workload's shape
    cfg = W.CONFIGS["plain_gpu"]
    K, M, B = cfg.K, cfg.M, cfg.nblocks
    N = K * M
    S_h, taps_h = W.make_uniform(cfg)
    S = torch.from_numpy(S_h).to(dev)
    taps = torch.from_numpy(taps_h).to(dev)
    d = torch.empty((B, K), dtype=torch.complex64, device=dev)
    db = torch.from_numpy(W.cn01(np.random.default_rng(10), (B, K)).astype(np.complex64)).to(dev)
    sb = torch.empty_like(S)
    # rotating copies of the large operands (about 0.5 GB in all), so that a step does not
    # find the previous step's data in the 256 MB last-level cache
    dsets = [(S, sb)] + [(S.clone(), torch.empty_like(S)) for _ in range(3)]

    def decstep(i):
        Si, sbi = dsets[i % len(dsets)]
        T.transform_decimated(Si, taps, K, M, out=d)
        T.transform_decimated_adjoint(db, taps, K, M, out=sbi)

    t = _timeit(decstep, steps)
    byts = (16.0 * N + 16.0 * K) * B
    idx = np.array([0, 2048, 4095])
    T.transform_decimated(S, taps, K, M, out=d)
    res["decimated"] = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
                        "achieved_GBps": round(byts / t / 1e9, 1),
                        "frac_hbm_peak": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
                        "rel_l2_forward": _rel(d.cpu().numpy()[idx], O.decimated(S_h[idx], taps_h, K)),
                        "workload": "eq. (7) on 4096 blocks K=128 M=15: forward (N -> K) + adjoint (K -> N)"}
    del S, taps, d, db, sb, dsets

    # ---- differentiation workload: forward + adjoint with the shared tap gradient
    cfg = W.CONFIGS["differentiation"]
    K, M, B = cfg.K, cfg.M, cfg.nblocks
    N = K * M
    S_h, taps_h = W.make_uniform(cfg)
    S = torch.from_numpy(S_h).to(dev)
    taps = torch.from_numpy(taps_h).to(dev)
    yb = torch.from_numpy(W.cn01(np.random.default_rng(9), (B, N)).astype(np.complex64)).to(dev)
    y = torch.empty_like(S)
    sb = torch.empty_like(S)
    tb = torch.empty(N, dtype=torch.float32, device=dev)

    # two buffer sets (0.6 GB each), alternated so that no step re-reads cached data
    S2, yb2 = S.clone(), yb.clone()
    y2, sb2 = torch.empty_like(S), torch.empty_like(S)
    dcalls = [(T.bind_forward(Si, taps, K, M, yi), T.bind_adjoint(ybi, taps, K, M, sbi, coeffs=Si, taps_bar=tb))
              for (Si, yi, ybi, sbi) in ((S, y, yb, sb), (S2, y2, yb2, sb2))]

    def dstep(i):
        df, da = dcalls[i % 2]
        df()
        da()

    t = _timeit(dstep, steps)
    byts = (16.0 + 24.0) * N * B
    res["differentiation"] = {"blocks_per_s": round(B / t, 1), "ms_per_step": round(t * 1e3, 4),
                              "achieved_GBps": round(byts / t / 1e9, 1),
                              "frac_hbm_peak": round(byts / t / 1e9 / HBM_PEAK_GBS, 4),
                              "workload": "8192 blocks K=256 M=9, forward + adjoint with the "
                                          "deterministic shared tap-gradient reduction"}

    # ---- non-iterative type-5 / type-4 methods: 256 problems of P = 1024 jittered
    #      instants, eta = 6, truncation ratio mu = 1e-7 (eq. (49))
    from oracle import lagrange as LG
    from paper_1604_06236_amd import nufft as NU
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

        t = _timeit(nstep, max(3, steps // 10))
        e = {"solves_per_s": round(2 * B / t, 1), "ms_per_step": round(t * 1e3, 4)}
        if not gridding:
            # exact non-uniform sum terms per step: each method does eta P^2 (eq. (28)) + P^2
            # (eq. (16)) + P^2 (the weights' type-1 sum, or the type-2 evaluation of s(t_q)),
            # and the refinement repeats the last P^2 term twice more (residual, second pass)
            terms = 2 * B * ((eta + 2) * P * P + (2 * P * P if refine else 0))
            e["nudft_terms_per_s"] = float(f"{terms / t:.4g}")
        r5 = (LG.type5_refined(t_h[0], s_h[0], eta, a, st) if refine else S_ref)
        r4 = (LG.type4_refined(t_h[0], A_h[0], eta, a, st) if refine else a_ref)
        e["rel_l2_type5_vs_oracle"] = _rel(S5.cpu().numpy()[0], r5)
        e["rel_l2_type4_vs_oracle"] = _rel(a4.cpu().numpy()[0], r4)
        e["rel_l2_type5_vs_gaussian_elimination"] = _rel(S5.cpu().numpy()[0], S_ge)
        nres[name] = e
        del ws
    # the same two solves from one shared setup (the instants-only part computed once)
    for name, gridding in (("exact_sums_shared_setup", False), ("gridding_shared_setup", True)):
        ws = torch.empty(NU.nufft_workspace_size(B, P, eta, NU.NUFFT_GRIDDING if gridding else 0),
                         dtype=torch.uint8, device=dev)

        def sstep(i, ws=ws, gridding=gridding):
            NU.nufft_setup(tt, eta, a, workspace=ws, gridding=gridding)
            NU.nufft_apply(5, tt, s, eta, a, ws, out=S5, gridding=gridding)
            NU.nufft_apply(4, tt, A, eta, a, ws, out=a4, gridding=gridding)

        t = _timeit(sstep, max(3, steps // 10))
        nres[name] = {"solves_per_s": round(2 * B / t, 1), "ms_per_step": round(t * 1e3, 4),
                      "rel_l2_type5_vs_oracle": _rel(S5.cpu().numpy()[0], S_ref),
                      "rel_l2_type4_vs_oracle": _rel(a4.cpu().numpy()[0], a_ref)}
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
                     "note": "executed FP64 MFMA work; a pure 16x16x4f64 MFMA loop sustains about 49 TFLOP/s"}}
    del zt
    res["nufft"] = nres
    return res


def cpu_baseline(S_h, taps_h, seconds):
    """The FP64 oracle (plain O(N^2) C, OpenMP over blocks) on a bounded sample of
    the same workload: forward + adjoint over the batch, repeated until about
    `seconds` of wall time have been spent."""
    import numpy as np
    from oracle import oracle as O
    O.build()
    nth = O.max_threads()
    B = S_h.shape[0]
    # calibrate on one block per thread
    t0 = time.perf_counter()
    y = O.forward(S_h[:nth], taps_h)
    O.adjoint(y, taps_h)
    per_block = (time.perf_counter() - t0) / nth
    target = max(nth, int(seconds / max(per_block, 1e-9)))
    done, dt = 0, 0.0
    t0 = time.perf_counter()
    while done < target:
        nb = min(B, target - done)
        y = O.forward(S_h[:nb], taps_h)
        O.adjoint(y, taps_h)
        done += nb
    dt = time.perf_counter() - t0
    return {"value": round(done / dt, 2), "unit": "blocks/s", "cores": nth, "kind": "oracle",
            "sample": f"{done} blocks of the K=128, M=15 batch (the batch repeated as needed), "
                      f"forward + adjoint, FP64 O(N^2), {dt:.1f} s on {nth} threads"}


if __name__ == "__main__":
    main()

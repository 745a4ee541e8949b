#!/usr/bin/env python3
"""Throughput of the FMM-based NUFFT + INUFFT on one MI355X.

One step = one forward transform (problem i, N = M = 2^20, y iid uniform on
[0, 2 pi)) plus one inverse transform (problem ii, N = M = 2^20, jittered
grid y_j = 2 pi (j + u_j)/N, u_j ~ U(-0.4, 0.4)), each one-shot (nufft_fwd,
inufft): setup of the data structure (Section 3.3) and evaluation.  Inputs are resident in HBM
before the timed region.  value = (N + M) / step time, i.e. points per
second for the forward + inverse pair.  The plain FP64 path (eps 1e-12) is
the headline; the mixed path (eps 1e-6) is timed on the same inputs.

Prints one JSON line.  Options: --steps K --warmup W --gpus 1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "(N+M)/s at rel-ℓ2 1e-12 (FP64) vs 1e-6 (mixed), N=M=2^20 fwd+inv"
PEAK_FP64 = 78.6e12      # MI355X FP64 vector (and matrix) FLOP/s
PEAK_FP32 = 157.3e12     # MI355X FP32 vector FLOP/s
PEAK_HBM = 8.0e12        # B/s
# HBM bytes per launch of the downward kernels from FETCH_SIZE and WRITE_SIZE
# (rocprofv3 --pmc, one counter per run), each scaled by what the counter
# reads for a plain 256 MiB elementwise kernel (fetch x2.000, write x1.000).
# Valid only for the kernel sources they were taken on: any change to them
# turns the figure back into null until the counters are taken again.
TRAFFIC = {
    "k_down_trans<double,cot,uniform sources,forward>": {
        "src_sha256": "813c8cdda1b43705f052e8d12d159b483bae82577d2b0f8752f7dc988c2d4398",
        "fetch": 33628461, "write": 8388600, "summary": "profiles/bench_kernels_2p20_traffic.txt"},
    "k_down_eval<double,cot,uniform sources,forward>": {
        "src_sha256": "813c8cdda1b43705f052e8d12d159b483bae82577d2b0f8752f7dc988c2d4398",
        "fetch": 44498491, "write": 34097133, "summary": "profiles/bench_kernels_2p20_traffic.txt"},
    "k_down_trans<double,cot,sorted sources,inverse>": {
        "src_sha256": "813c8cdda1b43705f052e8d12d159b483bae82577d2b0f8752f7dc988c2d4398",
        "fetch": 66970646, "write": 16777200, "summary": "profiles/bench_kernels_2p20_traffic.txt"},
    "k_down_eval<double,cot,sorted sources,inverse>": {
        "src_sha256": "813c8cdda1b43705f052e8d12d159b483bae82577d2b0f8752f7dc988c2d4398",
        "fetch": 64063607, "write": 16777200, "summary": "profiles/bench_kernels_2p20_traffic.txt"},
    "k_down_trans<double,log,sorted sources,log-sums>": {
        "src_sha256": "813c8cdda1b43705f052e8d12d159b483bae82577d2b0f8752f7dc988c2d4398",
        "fetch": 33863829, "write": 8388600, "summary": "profiles/bench_kernels_2p20_traffic.txt"},
    "k_down_eval<double,log,sorted sources,log-sums>": {
        "src_sha256": "813c8cdda1b43705f052e8d12d159b483bae82577d2b0f8752f7dc988c2d4398",
        "fetch": 32920440, "write": 25199584, "summary": "profiles/bench_kernels_2p20_traffic.txt"},
}
PHASES = ("fwd_plan_ms", "fwd_up_ms", "fwd_trans_ms", "fwd_eval_ms", "inv_plan_ms",
          "inv_up_ms", "inv_trans_ms", "inv_eval_ms", "log_up_ms", "log_trans_ms",
          "log_eval_ms")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the clustered-forward and batched figures")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain elementwise kernel that reads and "
                         "writes 256 MiB (known byte counts for scaling "
                         "memory-traffic counters)")
    return ap.parse_args()


def kernel_sources_sha256():
    import hashlib
    d = os.path.join(ROOT, "paper_1611_09379_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_of(kernel):
    t = TRAFFIC.get(kernel)
    if t is None or t["src_sha256"] != kernel_sources_sha256():
        return None
    return t["fetch"] + t["write"]


def trans_flops(info):
    """Algorithmic flops of one downward-translation launch (cot FMM, complex
    data, real operators): per box of levels 3..lmax one triangular L2L
    (P(P+1)/2 complex-by-real multiply-adds, 4 flops each) and 3 M2L
    (P^2 each), i.e. 2P(P+1) + 12P^2."""
    P, l = info.nterms, info.lmax
    boxes = (1 << (l + 1)) - 8 if l >= 3 else 0
    return boxes * (2 * P * (P + 1) + 12 * P * P)


def eval_flops(info, n_targets, n_sources):
    """Algorithmic flops of one evaluation launch: 3 N_t N_s / 2^lmax
    near-field pairs (Eq. 23) at 6 flops (difference, reciprocal,
    complex-by-real multiply-add) and a P-term complex Horner L2P (4 flops
    per term) per target."""
    P, l = info.nterms, info.lmax
    return 3.0 * n_targets * n_sources / (1 << l) * 6.0 + n_targets * 4.0 * P


def log_trans_flops(lmax, P):
    """The translations of the log-sum FMM: real data, so half the complex
    count of trans_flops: P(P+1) + 6P^2 per box of levels 3..lmax."""
    boxes = (1 << (lmax + 1)) - 8 if lmax >= 3 else 0
    return boxes * (P * (P + 1) + 6 * P * P)


def log_eval_flops(lmax, P, n):
    """The log-sum evaluation at its 2n targets (the n uniform points and the
    n sources): 3 (2n) n / 2^lmax near-field pairs (Eq. 23) at 3 flops
    (integer and fractional differences, product) and a P-term real Horner
    L2P (2 flops per term) per target."""
    return 3.0 * (2 * n) * n / (1 << lmax) * 3.0 + 2 * n * 2.0 * P


def run_path(fn, torch, N, M, yu, f, yj, gj, eps, steps, warmup):
    """Times `steps` one-shot fwd + inv pairs (nufft_fwd + inufft, one
    synchronisation each), then the same transforms through plans with
    events around the two kernels of each execute, and execute-only."""
    dt = f.dtype
    g = torch.empty(M, dtype=dt, device="cuda")
    fo = torch.empty(N, dtype=dt, device="cuda")
    dtc = fn.FN_C128 if dt == torch.complex128 else fn.FN_C64

    def one_step():
        fn.nufft_fwd(yu, f, eps, out=g)
        fn.inufft(yj, gj, eps, out=fo)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # phases: events on the library's stream (torch's current stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    ph = {k: [] for k in ("fwd_up", "fwd_trans", "fwd_eval", "inv_up", "inv_trans",
                          "inv_eval", "fwd_plan", "inv_plan", "log_up", "log_trans",
                          "log_eval")}
    log_terms = 0
    info_f = info_i = None
    for it in range(warmup + steps):
        t = time.perf_counter()
        pf = fn.Plan.forward(N, yu, eps, dtc)
        tpf = time.perf_counter() - t
        ev[0].record()
        pf.execute_phase(f, g, 0)
        ev[1].record()
        pf.execute_phase(f, g, 1)
        ev[2].record()
        pf.execute_phase(f, g, 2)
        ev[3].record()
        info_f = pf.info()
        pf.destroy()
        # the inverse setup's log-sum FMM is timed by the library's own
        # events (its kernels run inside the plan)
        fn.set_timing(True)
        t = time.perf_counter()
        pi = fn.Plan.inverse(yj, eps, dtc)
        tpi = time.perf_counter() - t
        fn.set_timing(False)
        tl = pi.timings()
        log_terms = tl["log_terms"]
        ev[4].record()
        pi.execute_phase(gj, fo, 0)
        ev[5].record()
        pi.execute_phase(gj, fo, 1)
        ev[6].record()
        pi.execute_phase(gj, fo, 2)
        ev[7].record()
        info_i = pi.info()
        pi.destroy()
        if it >= warmup:
            ph["fwd_up"].append(ev[0].elapsed_time(ev[1]))
            ph["fwd_trans"].append(ev[1].elapsed_time(ev[2]))
            ph["fwd_eval"].append(ev[2].elapsed_time(ev[3]))
            ph["inv_up"].append(ev[4].elapsed_time(ev[5]))
            ph["inv_trans"].append(ev[5].elapsed_time(ev[6]))
            ph["inv_eval"].append(ev[6].elapsed_time(ev[7]))
            ph["fwd_plan"].append(tpf * 1e3)
            ph["inv_plan"].append(tpi * 1e3)
            ph["log_up"].append(tl["log_up_ms"])
            ph["log_trans"].append(tl["log_trans_ms"])
            ph["log_eval"].append(tl["log_eval_ms"])

    # evaluation only (plan reused, Section 3.3), outside the headline
    pf = fn.Plan.forward(N, yu, eps, dtc)
    pi = fn.Plan.inverse(yj, eps, dtc)
    for _ in range(2):
        pf(f, g)
        pi(gj, fo)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        pf(f, g)
        pi(gj, fo)
    torch.cuda.synchronize()
    exec_wall = time.perf_counter() - t1
    pf.destroy()
    pi.destroy()
    # outputs of the timed one-shot transforms
    one_step()
    torch.cuda.synchronize()
    return {
        "wall_s": wall, "ms_per_step": 1e3 * wall / steps,
        "exec_ms_per_step": 1e3 * exec_wall / steps,
        **{k + "_ms": float(np.median(v) if k.endswith("plan") else np.mean(v))
           for k, v in ph.items()},
        "info_f": info_f, "info_i": info_i, "g": g, "fo": fo, "log_terms": log_terms,
    }


def run_batched(fn, torch, workloads, steps, warmup):
    """512 independent forward transforms, N_i log-uniform in [2^8, 2^16],
    M_i = rint(N_i U(0.5, 2)), uniform y: one-shot batched calls (setup and
    evaluation) and evaluation-only graph replays of a batch plan, for both
    precision paths, with depth and expansion length autotuned per size
    class first.  Throughput = (sum N_i + sum M_i) / time."""
    Ns, Ms = workloads.batched_sizes(512, seed=0)
    ys, fs = [], []
    for t, (N, M) in enumerate(zip(Ns, Ms)):
        y, f, c = workloads.forward_case(int(N), int(M), "uniform", seed=t)
        ys.append(torch.from_numpy(y).cuda())
        fs.append(torch.from_numpy(f).cuda())
    pts = int(Ns.sum() + Ms.sum())
    out = {"transforms": 512, "sum_N": int(Ns.sum()), "sum_M": int(Ms.sum())}
    # size classes lg = round(log2 sqrt(N M)) present, each with its median member
    lg = np.rint(0.5 * np.log2(Ns.astype(float) * Ms.astype(float))).astype(int)
    reps = {}
    for c in sorted(set(lg.tolist())):
        idx = np.nonzero(lg == c)[0]
        i = idx[np.argsort(Ns[idx])[len(idx) // 2]]
        reps[c] = (int(Ns[i]), int(Ms[i]))
    for name, dt, eps in (("f64", torch.complex128, 1e-12), ("mixed", torch.complex64, 1e-6)):
        dtc = fn.FN_C128 if dt == torch.complex128 else fn.FN_C64
        # autotuned depth and expansion length per size class (outside timing)
        t = time.perf_counter()
        tuned = {str(c): fn.autotune("fwd", n, m, eps, dtc) for c, (n, m) in reps.items()}
        tune_s = time.perf_counter() - t
        fx = [f.to(dt) for f in fs]
        gs = [torch.empty(y.shape[0], dtype=dt, device="cuda") for y in ys]
        for _ in range(warmup):
            fn.nufft_fwd_batched(ys, fx, eps, outs=gs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn.nufft_fwd_batched(ys, fx, eps, outs=gs)
        torch.cuda.synchronize()
        one = (time.perf_counter() - t) / steps
        b = fn.Batch.forward(ys, [int(n) for n in Ns], eps, dtc)
        for _ in range(warmup):
            b(fx, gs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            b(fx, gs)
        torch.cuda.synchronize()
        ex = (time.perf_counter() - t) / steps
        b.destroy()
        fn.autotune_clear()
        out[name] = {"eps": eps, "one_shot_ms": one * 1e3, "one_shot_points_per_s": pts / one,
                     "graph_exec_ms": ex * 1e3, "graph_exec_points_per_s": pts / ex,
                     "autotuned_lmax_nterms_by_size_class": tuned,
                     "autotune_s": tune_s}
    return out


def run_clustered(fn, torch, workloads, N, steps, warmup):
    """Forward transform on clustered targets (wrapped mixture of 8 Gaussians,
    sigma = 0.01), N = M, one-shot, both precision paths."""
    y, f, c = workloads.forward_case(N, N, "clustered", seed=0)
    yd = torch.from_numpy(y).cuda()
    f64 = torch.from_numpy(f).cuda()
    out = {"N": N, "M": N}
    for name, dt, eps in (("f64", torch.complex128, 1e-12), ("mixed", torch.complex64, 1e-6)):
        fx = f64.to(dt)
        g = torch.empty(N, dtype=dt, device="cuda")
        for _ in range(warmup):
            fn.nufft_fwd(yd, fx, eps, out=g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn.nufft_fwd(yd, fx, eps, out=g)
        torch.cuda.synchronize()
        dtm = (time.perf_counter() - t) / steps
        out[name] = {"eps": eps, "ms": dtm * 1e3, "points_per_s": 2 * N / dtm}
    return out


def cpu_baseline(N, M, yu, f, yj, seconds):
    """The oracle (direct sums, unchanged) on a bounded sample of the same
    workload, extrapolated to the full transforms: forward cost per target
    = one O(N) direct sum (Eq. p4); inverse cost per output = the two O(N)
    log-sums behind Eq. (p8) plus one O(N) cot sum (Eq. p6)."""
    import oracle
    cores = oracle.threads()
    rng = np.random.default_rng(7)
    # calibrate on a small sample, then size the sample to ~seconds of work
    s0 = max(cores, 32)
    t = time.perf_counter()
    oracle.fwd_at(N, yu, f, rng.choice(M, s0, replace=False))
    per_f = (time.perf_counter() - t) / s0
    t = time.perf_counter()
    oracle.logsums(N, yj, ks=rng.choice(N, s0, replace=False),
                   js=rng.choice(N, s0, replace=False))
    per_i = (time.perf_counter() - t) / s0 + per_f
    S = int(max(s0, min(M, seconds / (per_f + per_i))))
    sel_f = rng.choice(M, S, replace=False)
    sel_i = rng.choice(N, S, replace=False)
    t = time.perf_counter()
    oracle.fwd_at(N, yu, f, sel_f)
    tf = time.perf_counter() - t
    t = time.perf_counter()
    oracle.logsums(N, yj, ks=sel_i, js=sel_i)
    oracle.fwd_at(N, yj, f, sel_i)      # same O(N) cot sum per output
    ti = time.perf_counter() - t
    t_pair = tf * M / S + ti * N / S
    return {"value": (N + M) / t_pair, "unit": "points/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{S} forward targets + {S} inverse outputs (log-sums "
                      f"and cot sum) of the N=M=2^{int(np.log2(N))} workload, "
                      f"{tf + ti:.1f} s measured, extrapolated linearly to all "
                      f"N + M outputs ({t_pair:.0f} s per fwd+inv pair)"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1611_09379_amd as fn
    import workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    fn.load_library()
    if args.calibrate_copy:
        # a plain elementwise kernel: reads 256 MiB, writes 256 MiB
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    N = M = 1 << args.log2n
    yu_h, f_h, c_h = workloads.forward_case(N, M, "uniform", seed=0)
    yj_h, cj_h = workloads.inverse_case(N, 0.4, seed=1)
    yu = torch.from_numpy(yu_h).cuda()
    yj = torch.from_numpy(yj_h).cuda()
    f64 = torch.from_numpy(f_h).cuda()
    # inverse input: samples of the same band-limited function at the jittered
    # points (computed once, before timing)
    gj64 = fn.nufft_fwd(yj, f64, 1e-12)
    torch.cuda.synchronize()

    res = run_path(fn, torch, N, M, yu, f64, yj, gj64, 1e-12, args.steps, args.warmup)
    # accuracy of the timed outputs (outside the timed region)
    sel = np.random.default_rng(3).choice(M, 64, replace=False)
    g_h = res["g"].cpu().numpy()
    fo_h = res["fo"].cpu().numpy()
    acc = {"inv_roundtrip_rel_l2": float(np.linalg.norm(fo_h - f_h) / np.linalg.norm(f_h))}
    if not args.no_cpu_baseline:
        import oracle
        ref = oracle.fwd_at(N, yu_h, f_h, sel)
        acc["fwd_rel_l2_vs_oracle_64"] = float(np.linalg.norm(g_h[sel] - ref) / np.linalg.norm(ref))

    info_f, info_i = res["info_f"], res["info_i"]
    # dominant kernel: the longest of the downward translation and evaluation
    # kernels of the two transforms and of the inverse setup's log-sum FMM
    # (each timed alone with events)
    cands = [
        ("k_down_trans<double,cot,uniform sources,forward>", "mfma", trans_flops(info_f),
         res["fwd_trans_ms"]),
        ("k_down_eval<double,cot,uniform sources,forward>", "alu",
         eval_flops(info_f, M, N), res["fwd_eval_ms"]),
        ("k_down_trans<double,cot,sorted sources,inverse>", "mfma", trans_flops(info_i),
         res["inv_trans_ms"]),
        ("k_down_eval<double,cot,sorted sources,inverse>", "alu",
         eval_flops(info_i, N, N), res["inv_eval_ms"]),
        ("k_down_trans<double,log,sorted sources,log-sums>", "mfma",
         log_trans_flops(info_i.lmax, res["log_terms"]), res["log_trans_ms"]),
        ("k_down_eval<double,log,sorted sources,log-sums>", "alu",
         log_eval_flops(info_i.lmax, res["log_terms"], N), res["log_eval_ms"]),
    ]
    dom, bound, fl, dur_ms = max(cands, key=lambda c: c[3])
    dur = dur_ms * 1e-3
    roof = {"bound": bound, "achieved": fl / dur / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": fl / dur / PEAK_FP64, "traffic": traffic_of(dom), "traffic_unit": "bytes per launch",
            "kernel": dom, "flops_per_launch": fl, "avg_launch_ms": dur_ms,
            "others": {c[0]: {"bound": c[1], "tflops": c[2] / (c[3] * 1e-3) / 1e12,
                              "frac": c[2] / (c[3] * 1e-3) / PEAK_FP64, "ms": c[3],
                              "traffic": traffic_of(c[0])}
                       for c in cands}}

    out = {
        "metric": METRIC,
        "value": (N + M) / (res["ms_per_step"] * 1e-3),
        "unit": "points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"fwd uniform y + inv jittered grid (u~U(-0.4,0.4)), "
                               f"N=M=2^{args.log2n}, one-shot, FP64 eps=1e-12",
                   "N": N, "M": M, "eps": 1e-12,
                   "fwd": {"p": info_f.p, "q": info_f.q, "lmax": info_f.lmax,
                           "nterms": info_f.nterms},
                   "inv": {"p": info_i.p, "q": info_i.q, "lmax": info_i.lmax,
                           "nterms": info_i.nterms}},
        "phases_ms": {k: round(res[k], 4) for k in PHASES},
        "exec_only": {"ms_per_step": res["exec_ms_per_step"],
                      "value": (N + M) / (res["exec_ms_per_step"] * 1e-3)},
        "accuracy": acc,
        "roofline": roof,
    }
    if not args.no_mixed:
        f32 = f64.to(torch.complex64)
        gj32 = gj64.to(torch.complex64)
        rm = run_path(fn, torch, N, M, yu, f32, yj, gj32, 1e-6, args.steps, args.warmup)
        fo_m = rm["fo"].cpu().numpy()
        mixed = {"value": (N + M) / (rm["ms_per_step"] * 1e-3),
                 "ms_per_step": rm["ms_per_step"], "dtype": "mixed f32/f64",
                 "eps": 1e-6,
                 "speedup_vs_f64": res["ms_per_step"] / rm["ms_per_step"],
                 "exec_only_ms_per_step": rm["exec_ms_per_step"],
                 "phases_ms": {k: round(rm[k], 4) for k in PHASES},
                 "inv_roundtrip_rel_l2": float(np.linalg.norm(fo_m - f_h) / np.linalg.norm(f_h))}
        if not args.no_cpu_baseline:
            import oracle
            gm = rm["g"].cpu().numpy()
            ref = oracle.fwd_at(N, yu_h, f32.cpu().numpy().astype(np.complex128), sel)
            mixed["fwd_rel_l2_vs_oracle_64"] = float(np.linalg.norm(gm[sel] - ref) / np.linalg.norm(ref))
        out["mixed"] = mixed
    if not args.no_extra:
        out["forward_clustered"] = run_clustered(fn, torch, workloads, N, args.steps,
                                                 args.warmup)
        out["batched_512"] = run_batched(fn, torch, workloads, args.steps, args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N, M, yu_h, f_h, yj_h, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

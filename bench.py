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
PEAK_FP64 = 78.6e12      # MI355X FP64 vector and matrix FLOP/s
PEAK_FP32 = 157.3e12     # MI355X FP32 vector and matrix FLOP/s
PEAK_HBM = 8.0e12        # B/s
# HBM bytes per launch of each phase, from FETCH_SIZE and WRITE_SIZE
# (rocprofv3 --pmc, one counter per run) summed over the phase's kernels,
# each scaled by what the counter reads for a plain 256 MiB elementwise
# kernel (fetch x2.000, write x1.000).  Valid only for the kernel sources
# they were taken on: any change to them turns the figure back into null
# until the counters are taken again.
TRAFFIC_SRC_SHA256 = "ebab5fe67d7837f5835498948b0e1918071ccbd08f3a72fe33f47d6194d1822c"
TRAFFIC = {
    "fwd_eval": 98108347,
    "fwd_eval_mixed": 83496503,
    "fwd_sort": 43198233,
    "fwd_trans": 64106987,
    "fwd_trans_mixed": 16169026,
    "fwd_up": 43069235,
    "fwd_up_mixed": 17254794,
    "inv_eval": 80831641,
    "inv_eval_mixed": 50438550,
    "inv_sort": 87198624,
    "inv_trans": 127789969,
    "inv_trans_mixed": 32160461,
    "inv_up": 142067037,
    "inv_up_mixed": 81920039,
    "log_eval": 58107486,
    "log_trans": 64382847,
    "log_up": 43753418,
    "log_up_mixed": 34979643,
}
# phase keys of one step (ms): plan wall time, then each measured phase
PHASES = ("fwd_plan_ms", "fwd_sort_ms", "fwd_up_ms", "fwd_trans_ms", "fwd_eval_ms",
          "inv_plan_ms", "inv_sort_ms", "log_up_ms", "log_trans_ms", "log_eval_ms",
          "inv_up_ms", "inv_trans_ms", "inv_eval_ms")


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
    ap.add_argument("--study", choices=("cond", "eps_th"), default=None,
                    help="instead of the benchmark: the inverse's conditioning "
                         "study (cond) or the precision floor eps_th(N) study")
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


def traffic_of(phase, mixed=False):
    """Calibrated HBM bytes of one launch of the phase's kernels (null when
    not taken on the current kernel sources).  The mixed path's entries end
    in _mixed; its sorts and log-sums run the binary64 kernels."""
    if TRAFFIC_SRC_SHA256 != kernel_sources_sha256():
        return None
    if mixed:
        t = TRAFFIC.get(phase + "_mixed")
        if t is None and phase.startswith(("log_", "fwd_sort", "inv_sort")):
            t = TRAFFIC.get(phase)
        return t
    return TRAFFIC.get(phase)


def boxes(l, lo=3):
    """Boxes of levels lo..l of the binary tree (2^lo + ... + 2^l)."""
    return (1 << (l + 1)) - (1 << lo) if l >= lo else 0


def trans_flops(l, P, complex_data=True):
    """Algorithmic flops of the downward translations: per box of levels
    3..l three M2L (P^2 multiply-adds each) and one triangular L2L
    (P(P+1)/2), 4 flops per multiply-add of a complex by a real, 2 for real
    data: 12 P^2 + 2 P(P+1) per box (complex), half that for the log-sums."""
    f = boxes(l) * (12 * P * P + 2 * P * (P + 1))
    return f if complex_data else f // 2


def eval_flops(l, P, n_targets, n_sources):
    """Algorithmic flops of one cot evaluation: 3 N_t N_s / 2^l near-field
    pairs (Eq. 23) at 6 flops (difference, reciprocal, complex-by-real
    multiply-add) and a P-term complex Horner L2P (4 flops per term) per
    target."""
    return 3.0 * n_targets * n_sources / (1 << l) * 6.0 + n_targets * 4.0 * P


def log_eval_flops(l, P, n):
    """The log-sum evaluation at its 2n targets (the n uniform points and the
    n sources): 3 (2n) n / 2^l near-field pairs (Eq. 23) at 3 flops
    (integer and fractional differences, product) and a P-term real Horner
    L2P (2 flops per term) per target."""
    return 3.0 * (2 * n) * n / (1 << l) * 3.0 + 2 * n * 2.0 * P


def up_bytes(l, PU, n, src_bytes, coef_bytes):
    """Algorithmic HBM bytes of an upward pass: the sources read once
    (src_bytes each: weights and, for sorted sources, grid units and leaf)
    and every multipole of levels 2..l written once (PU coefficients of
    coef_bytes per box)."""
    return n * src_bytes + boxes(l, 2) * PU * coef_bytes


def sort_bytes(n):
    """Algorithmic HBM bytes of a sort: y read once (8 B per point), the
    sorted point (grid units and index, 16 B) written once."""
    return 24.0 * n


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
                          "log_eval", "fwd_sort", "inv_sort")}
    log_terms = 0
    info_f = info_i = None
    for it in range(warmup + steps):
        fn.set_timing(True)   # events around the sort (and the log-sum FMM)
        t = time.perf_counter()
        pf = fn.Plan.forward(N, yu, eps, dtc)
        tpf = time.perf_counter() - t
        fn.set_timing(False)
        sort_f = pf.timings()["sort_ms"]
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
        sort_i = tl["sort_ms"]
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
            ph["fwd_sort"].append(sort_f)
            ph["inv_sort"].append(sort_i)
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


def run_adjoint(fn, torch, workloads, N, steps, warmup):
    """Adjoint transform f = K^H g (the type-1 direction), N = M, uniform y,
    one-shot, both precision paths."""
    y, f, c = workloads.forward_case(N, N, "uniform", seed=5)
    yd = torch.from_numpy(y).cuda()
    g64 = torch.from_numpy(f).cuda()      # any M values serve as the input
    out = {"N": N, "M": N}
    for name, dt, eps in (("f64", torch.complex128, 1e-12), ("mixed", torch.complex64, 1e-6)):
        gx = g64.to(dt)
        fo = torch.empty(N, dtype=dt, device="cuda")
        for _ in range(warmup):
            fn.nufft_adj(yd, gx, N, eps, out=fo)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn.nufft_adj(yd, gx, N, eps, out=fo)
        torch.cuda.synchronize()
        dtm = (time.perf_counter() - t) / steps
        out[name] = {"eps": eps, "ms": dtm * 1e3, "points_per_s": 2 * N / dtm}
    return out


def run_large(fn, torch, workloads, warmup=1, steps=3):
    """The large configuration: a forward transform at N = M = 2^24 (uniform
    y) and an inverse at N = 2^22 (jittered grid, u ~ U(-0.3, 0.3)), eps
    1e-10 (binary64) and 1e-6 (mixed): one-shot times and execute-only
    times (plans reused)."""
    out = {}
    Nf, Ni = 1 << 24, 1 << 22
    y, f, c = workloads.forward_case(Nf, Nf, "uniform", seed=11)
    yi, ci = workloads.inverse_case(Ni, 0.3, seed=12)
    rng = np.random.default_rng(13)
    gi = rng.standard_normal(Ni) + 1j * rng.standard_normal(Ni)
    yd, yid = torch.from_numpy(y).cuda(), torch.from_numpy(yi).cuda()
    f64, gi64 = torch.from_numpy(f).cuda(), torch.from_numpy(gi).cuda()
    del y, f, c, yi, ci, gi

    def timed(fun):
        for _ in range(warmup):
            fun()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fun()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    for name, dt, eps in (("f64", torch.complex128, 1e-10), ("mixed", torch.complex64, 1e-6)):
        fx, gx = f64.to(dt), gi64.to(dt)
        g = torch.empty(Nf, dtype=dt, device="cuda")
        fo = torch.empty(Ni, dtype=dt, device="cuda")
        tf = timed(lambda: fn.nufft_fwd(yd, fx, eps, out=g))
        ti = timed(lambda: fn.inufft(yid, gx, eps, out=fo))
        pf = fn.Plan.forward(Nf, yd, eps, fn.FN_C128 if dt == torch.complex128 else fn.FN_C64)
        pi = fn.Plan.inverse(yid, eps, fn.FN_C128 if dt == torch.complex128 else fn.FN_C64)
        ef = timed(lambda: pf.execute(fx, out=g))
        ei = timed(lambda: pi.execute(gx, out=fo))
        info_f, info_i = pf.info(), pi.info()
        pf.destroy()
        pi.destroy()
        out[name] = {"eps": eps,
                     "fwd_2p24": {"one_shot_ms": tf * 1e3, "points_per_s": 2 * Nf / tf,
                                  "exec_ms": ef * 1e3, "lmax": info_f.lmax,
                                  "nterms": info_f.nterms},
                     "inv_2p22": {"one_shot_ms": ti * 1e3, "points_per_s": 2 * Ni / ti,
                                  "exec_ms": ei * 1e3, "lmax": info_i.lmax,
                                  "nterms": info_i.nterms}}
        del fx, gx, g, fo
    return out


def run_spectral(fn, torch, workloads, N, steps, warmup):
    """Spectral transforms (Eq. p1): coefficients -> values at uniform y
    (forward) and values at a jittered grid -> coefficients (inverse),
    N = M, both precision paths.  One-shot times, and the uniform DFT's
    share (rocFFT) as the difference between spectral and plain plan
    executes on the same points, timed with events."""
    y, f, c = workloads.forward_case(N, N, "uniform", seed=7)
    yj, cj = workloads.inverse_case(N, 0.4, seed=8)
    yd, yjd = torch.from_numpy(y).cuda(), torch.from_numpy(yj).cuda()
    c64 = torch.from_numpy(c).cuda()
    out = {"N": N, "M": N}
    for name, dt, eps in (("f64", torch.complex128, 1e-12), ("mixed", torch.complex64, 1e-6)):
        dtc = fn.FN_C128 if dt == torch.complex128 else fn.FN_C64
        cx = c64.to(dt)
        g = torch.empty(N, dtype=dt, device="cuda")
        co = torch.empty(N, dtype=dt, device="cuda")
        fn.nufft_spec_fwd(yd, cx, eps, out=g)
        gj = fn.nufft_spec_fwd(yjd, cx, eps)
        for _ in range(warmup):
            fn.nufft_spec_fwd(yd, cx, eps, out=g)
            fn.inufft_spec(yjd, gj, eps, out=co)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn.nufft_spec_fwd(yd, cx, eps, out=g)
            fn.inufft_spec(yjd, gj, eps, out=co)
        torch.cuda.synchronize()
        one = (time.perf_counter() - t) / steps
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

        def timed(plan, x, o):
            for _ in range(2):
                plan(x, o)
            ev[0].record()
            for _ in range(steps):
                plan(x, o)
            ev[1].record()
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1]) / steps

        pf, psf = fn.Plan.forward(N, yd, eps, dtc), fn.Plan.spectral_forward(N, yd, eps, dtc)
        pi, psi = fn.Plan.inverse(yjd, eps, dtc), fn.Plan.spectral_inverse(yjd, eps, dtc)
        tf, tsf = timed(pf, cx, g), timed(psf, cx, g)
        ti, tsi = timed(pi, gj, co), timed(psi, gj, co)
        for p_ in (pf, psf, pi, psi):
            p_.destroy()
        out[name] = {"eps": eps, "one_shot_fwd_plus_inv_ms": one * 1e3,
                     "points_per_s": 2 * N / one,
                     "exec_fwd_ms": tsf, "exec_inv_ms": tsi,
                     "dft_fwd_ms": tsf - tf, "dft_inv_ms": tsi - ti}
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


def phase_table(res, N, M, mixed):
    """Every measured phase of one step: (key, kernels, bound, work, unit,
    peak).  Work is algorithmic: flops for the matrix-core translations
    and the vector evaluations, HBM bytes for the sorts, upward passes and
    weights (the kernels and their counts are listed in the design notes).
    The mixed path's cot translations and evaluations are priced against
    the binary32 peaks, everything in binary64 against the binary64 ones."""
    fi, ii = res["info_f"], res["info_i"]
    cb = 8 if mixed else 16                  # bytes of one complex value
    pk = PEAK_FP32 if mixed else PEAK_FP64
    lf, li = fi.lmax, ii.lmax
    T = "TFLOP/s"
    return [
        ("fwd_sort", "k_hist k_colscan k_scan_work k_place_rec", "hbm", sort_bytes(M), "GB/s", PEAK_HBM),
        ("fwd_up", "k_up_band (P2M, M2M)", "hbm", up_bytes(lf, fi.mterms, N, cb, cb), "GB/s", PEAK_HBM),
        ("fwd_trans", "k_m2l k_down_trans", "mfma", trans_flops(lf, fi.nterms), T, pk),
        ("fwd_eval", "k_down_eval (forward)", "alu", eval_flops(lf, fi.nterms, M, N), T, pk),
        ("inv_sort", "k_hist k_colscan k_scan_work k_place_rec k_leaf_order", "hbm", sort_bytes(N), "GB/s", PEAK_HBM),
        ("log_up", "k_up_band (log-sums)", "hbm", up_bytes(li, ii.log_mterms, N, 16, 8), "GB/s", PEAK_HBM),
        ("log_trans", "k_m2l k_down_trans (log-sums)", "mfma",
         trans_flops(li, ii.log_nterms, complex_data=False), T, PEAK_FP64),
        ("log_eval", "k_down_eval (log-sums, Chat, Dhat)", "alu",
         log_eval_flops(li, ii.log_nterms, N), T, PEAK_FP64),
        ("inv_up", "k_weights k_up_band (inverse)", "hbm",
         N * (16 + 2 * cb + 4) + up_bytes(li, ii.mterms, N, cb + 16, cb), "GB/s", PEAK_HBM),
        ("inv_trans", "k_m2l k_down_trans (inverse)", "mfma", trans_flops(li, ii.nterms), T, pk),
        ("inv_eval", "k_down_eval (inverse)", "alu", eval_flops(li, ii.nterms, N, N), T, pk),
    ]


def roofline(res, N, M, mixed):
    """The dominant kernel (the longest phase that is a single kernel; the
    sorts, upward passes and translations take several launches) with its
    fraction of the roof that bounds it, and every phase under `others`."""
    rows = {}
    for key, kern, bound, work, unit, peak in phase_table(res, N, M, mixed):
        ms = res[key + "_ms"]
        rate = work / (ms * 1e-3)
        scale = 1e9 if unit == "GB/s" else 1e12
        rows[key] = {"kernels": kern, "bound": bound, "ms": ms,
                     "achieved": rate / scale, "peak": peak / scale, "unit": unit,
                     "frac": rate / peak, "work": work,
                     "work_unit": "bytes" if unit == "GB/s" else "flops",
                     "traffic": traffic_of(key, mixed)}
    dom = max((k for k in rows if len(rows[k]["kernels"].split()) == 1 or
               rows[k]["kernels"].startswith("k_down_eval")),
              key=lambda k: rows[k]["ms"])
    d = rows[dom]
    return {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
            "unit": d["unit"], "frac": d["frac"], "traffic": d["traffic"],
            "traffic_unit": "bytes per launch", "kernel": dom + ": " + d["kernels"],
            "work_per_launch": d["work"], "avg_launch_ms": d["ms"], "others": rows}


def study_cond(fn, torch, workloads):
    """The inverse across point distributions (Section 3: its error depends on
    the distribution of the points), N = 1024: the condition number of K
    (numpy), the range of the log-sums of Eq. (p8), the square inverse on
    both precision paths (status and error against the band-limited
    function whose exact values it inverts), and the least-squares inverse
    (CG on the normal equations) with M = N and with M = 4N points of the
    same distribution."""
    import oracle
    N = 1024
    rng = np.random.default_rng(0)
    c = workloads.coefficients(N, rng)
    f = workloads.samples_from_coefficients(c)

    def pts(kind, par, M, seed):
        r = np.random.default_rng(seed)
        if kind == "jitter":
            k = M // N
            base = np.concatenate([workloads.points_jittered(N, par, r) + 2 * np.pi * i / (k * N)
                                   for i in range(k)]) if k > 1 else workloads.points_jittered(N, par, r)
            return np.mod(base, 2 * np.pi)
        if kind == "uniform":
            return workloads.points_uniform(M, r)
        if kind == "gap":
            return 2 * np.pi * par * (np.arange(M) + r.uniform(-0.3, 0.3, M)) / M + 1e-3
        return workloads.points_clustered(M, r, sigma=par)

    cases = [("jitter", a) for a in (0.1, 0.25, 0.3, 0.4, 0.45, 0.49)] + [("uniform", 0)] + \
            [("gap", a) for a in (0.97, 0.9)] + [("clustered", s_) for s_ in (0.3, 0.1, 0.01)]
    rows = []
    for kind, par in cases:
        y = pts(kind, par, N, 1)
        g = oracle.fwd(N, y, f)
        row = {"points": kind, "param": par, "N": N}
        try:
            row["cond_K"] = float(np.linalg.cond(oracle.kmatrix(N, y)))
        except Exception:
            row["cond_K"] = None
        lC, _, lD, _ = oracle.logsums(N, y)
        row["max_abs_log_C_D"] = float(max(np.abs(lC[np.isfinite(lC)]).max(), np.abs(lD).max()))
        try:
            row["oracle_inv_err"] = float(np.linalg.norm(oracle.inv(N, y, g) - f) / np.linalg.norm(f))
        except oracle.OracleError as e:
            row["oracle_inv_err"] = str(e)
        for name, dt, eps in (("f64", torch.complex128, 1e-12), ("mixed", torch.complex64, 1e-6)):
            try:
                fo = fn.inufft(torch.from_numpy(y).cuda(), torch.from_numpy(g).cuda().to(dt), eps)
                row[f"inv_{name}_err"] = float(np.linalg.norm(fo.cpu().numpy() - f) / np.linalg.norm(f))
            except fn.NufftError as e:
                row[f"inv_{name}_err"] = fn.STATUS_NAMES[e.status]
        for mult in (1, 4):
            ym = pts(kind, par, mult * N, 2) if mult > 1 else y
            gm = oracle.fwd(N, ym, f)
            out, it, res = fn.nufft_lsq(torch.from_numpy(ym).cuda(), torch.from_numpy(gm).cuda(),
                                        N, 1e-12, tol=1e-12, maxiter=1000)
            row[f"lsq_M{mult}N"] = {"iters": it, "resid": res,
                                    "err": float(np.linalg.norm(out.cpu().numpy() - f) / np.linalg.norm(f))}
        print(json.dumps(row), flush=True)
        rows.append(row)
    return rows


def study_eps_th(fn, torch, workloads):
    """The precision floor of the binary64 path, eps_th(N) (Section 3.1): for
    f = 1 (exact g = 1, the paper's max-abs measure) and for random f
    (relative l2 against the oracle on sampled targets), the error at
    requested eps = 1e-8 ... 1e-15; eps_th(N) is the smallest error reached.
    p_th, q_th (Fig. comp6): the smallest explicit expansion length (16, 32,
    48; with q = 30) and regular-part truncation q (with p = 48) whose f = 1
    error stays within 1.25 eps_th(N); the Eq. (18.2) values at eps_th(N)
    beside them."""
    import oracle
    rows = []
    for L in (3, 6, 8, 10, 12, 14, 16, 18, 20):
        N = M = 1 << L
        rng = np.random.default_rng(L)
        y = workloads.points_uniform(M, rng)
        yd = torch.from_numpy(y).cuda()
        ones = torch.ones(N, dtype=torch.complex128, device="cuda")
        c = workloads.coefficients(N, rng)
        f = workloads.samples_from_coefficients(c)
        fd = torch.from_numpy(f).cuda()
        sel = rng.choice(M, min(M, 256), replace=False)
        ref = oracle.fwd_at(N, y, f, sel)

        def errs(eps, p=0, q=0):
            plan = fn.Plan.forward(N, yd, eps, fn.FN_C128, p=p, q=q)
            g1 = plan(ones).cpu().numpy()
            gr = plan(fd).cpu().numpy()
            info = plan.info()
            plan.destroy()
            return (float(np.abs(g1 - 1).max()),
                    float(np.linalg.norm(gr[sel] - ref) / np.linalg.norm(ref)), info)

        row = {"N": N, "by_eps": {}}
        best_one, best_rand = 1.0, 1.0
        for e in (1e-8, 1e-10, 1e-12, 1e-13, 1e-14, 1e-15):
            ea, er, info = errs(e)
            row["by_eps"][f"{e:g}"] = {"max_abs_err_f1": ea, "rel_l2_random": er,
                                       "nterms": info.nterms, "q": info.q}
            best_one, best_rand = min(best_one, ea), min(best_rand, er)
        by_q = {}
        for q in range(8, 31, 2):
            by_q[q] = errs(1e-15, p=48, q=q)[:2]
        by_p = {}
        for p in (16, 32, 48):
            by_p[p] = errs(1e-15, p=p, q=30)[:2]
        for v in list(by_q.values()) + list(by_p.values()):
            best_one, best_rand = min(best_one, v[0]), min(best_rand, v[1])
        q_th = min((q for q, v in by_q.items() if v[0] <= 1.25 * best_one), default=None)
        p_th = min((p for p, v in by_p.items() if v[0] <= 1.25 * best_one), default=None)
        p18, q18, l = fn.select_params(N, M, max(best_one, 1e-15))
        mach = errs(0.0)
        row.update({"eps_th_max_abs_f1": best_one, "eps_th_rel_l2_random": best_rand,
                    "p_th": p_th, "q_th": q_th, "eq18_2_at_eps_th": {"p": p18, "q": q18},
                    "by_q_p48": {str(k): v for k, v in by_q.items()},
                    "by_p_q30": {str(k): v for k, v in by_p.items()},
                    "machine_mode": {"max_abs_err_f1": mach[0], "rel_l2_random": mach[1],
                                     "nterms": mach[2].nterms, "q": mach[2].q,
                                     "eps_th_reported": mach[2].eps}})
        print(json.dumps(row), flush=True)
        rows.append(row)
    return rows


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
    if args.study:
        rows = (study_cond if args.study == "cond" else study_eps_th)(fn, torch, workloads)
        print(json.dumps({"study": args.study, "rows": rows}), flush=True)
        return
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
    roof = roofline(res, N, M, mixed=False)

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
                 "roofline": roofline(rm, N, M, mixed=True),
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
        out["adjoint"] = run_adjoint(fn, torch, workloads, N, args.steps, args.warmup)
        out["spectral"] = run_spectral(fn, torch, workloads, N, args.steps, args.warmup)
        out["batched_512"] = run_batched(fn, torch, workloads, args.steps, args.warmup)
        out["large"] = run_large(fn, torch, workloads)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(N, M, yu_h, f_h, yj_h, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

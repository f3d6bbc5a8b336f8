"""Throughput benchmark of the IRLS reconstruction on one MI355X.

One step = one whole reconstruction (every outer IRLS iteration: Gram matrix,
FP64 eigen-decomposition, weights, filter product, masks, CG) of the
256 x 256 x 20-echo workload with filter 15 x 15 x 5, 20 outer x 15 CG
iterations, on seeded synthetic data already resident in HBM.

Prints one JSON line: IRLS iterations/s; the roofline of the dominant
hand-written kernel (algorithmic bytes or flops per launch / measured launch
time, HIP events on the plan's stream); the CG iteration and the whole
reconstruction against the HBM roofline on the method's own bytes; latency
percentiles and solves/s of a short Poisson request stream and slices/s of a
batch of uneven slices; the FP64 CPU oracle timed on a bounded sample on the
host cores.  Other modes (--workload) print the line of one other workload;
--workload calib runs the plain device copy used to calibrate the HBM
counters under rocprofv3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes(kind: str, T: int, P: int, Q: int, M: int, N1: int, N2: int, nc: int = 0) -> float:
    """Bytes one launch of a kernel class must move (complex64 = 8 B per element).

    Units: V = T P Q volume elements; mask S 1 B per element; masks E
    W = M(M+1)/2 complex64 planes of P x Q; nc coils (0: single channel).
    """
    V = T * P * Q
    W = M * (M + 1) // 2
    s = N1 * N2 * M
    c = 8
    if kind == "rows":     # read r, p_old; write p and the row-transformed volume t
        return 4 * V * c
    if kind == "cols":     # read t (coils: the image rho) and the masks E; write t
        return 2 * V * c + W * P * Q * c
    if kind == "fin":      # read t, p, S (1 B); write q (coils: no S; the complex128 group
        if nc:             # sums of the coil combination instead)
            return 3 * V * c + min(nc, 4) * V * 16
        return 3 * V * c + V
    if kind == "coil":     # columns: read t and the maps, write rho and nc volumes (complex64);
        g = min(nc, 4)     # rows: read the nc volumes and S, write them in complex128;
        return ((2 + nc) * V * c + nc * P * Q * c     # combine: read the complex128 volumes and
                + nc * V * c + V + nc * V * 16        # the maps, write the group sums (complex128)
                + nc * V * 16 + nc * P * Q * c + g * V * 16)
    if kind == "update":   # read x, p, r, q; write x, r
        return 6 * V * c
    if kind == "gram":     # images (read x, write/read t, write img), read img, write R
        return 5 * V * c + s * s * 16
    if kind == "masks":    # read the lag sums (spectral path) or H (2 s^2 doubles); write E
        g = spectral_groups(N1, N2, M)
        lag = W * (2 * N1 - 1) * (2 * N2 - 1) * 16 if g else 2 * s * s * 8
        return lag + W * P * Q * c
    if kind == "filter":   # read U (s^2 complex128); write H (2 s^2 doubles)
        return s * s * 16 + 2 * s * s * 8
    if kind == "voxel":    # pixel-wise weights: read the images, write the masks (the masks
        return V * c + W * P * Q * c   # pass; FP64 Jacobi arithmetic per pixel sets its time)
    return 0.0


def spectral_groups(N1: int, N2: int, M: int) -> int:
    """Eigenvector groups of the spectral lag sums (0: the shape takes the H path);
    the same rule as the library's: M <= 5, 2 N1 - 1 <= 32, s <= 2048, 64 KB of LDS
    for the accumulation and the inverse transform, partial and slice sums within
    s^2 complex128."""
    s, W = N1 * N2 * M, M * (M + 1) // 2
    L1, L2 = 2 * N1 - 1, 2 * N2 - 1
    if M > 5 or L1 > 32 or s > 2048:
        return 0
    if (s + M * N1 * 8 + L1 + L2) * 16 > 65536 or (2 * L1 * L2 + L1 + L2) * 16 > 65536:
        return 0
    gmax = (s * s) // (W * L1 * L2) - 8
    if gmax < 1:
        return 0
    g = min(gmax, 128, s)
    kper = -(-s // g)
    return -(-s // kper)


def spectral_flop(N1: int, N2: int, M: int) -> float:
    """Flops of the spectral lag sums (complex MAC = 8 flop): per eigenvector the
    N2-point DFTs of its M N1 rows at L2 frequencies, the N1-point DFTs of the
    M L1 L2 outputs, and W pair products at each of the L1 L2 frequencies."""
    s, W = N1 * N2 * M, M * (M + 1) // 2
    L1, L2 = 2 * N1 - 1, 2 * N2 - 1
    return 8.0 * s * (M * N1 * L2 * N2 + M * L1 * L2 * N1 + W * L1 * L2)


FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix
FP64_VALU_PEAK_TFLOPS = 78.6  # 256 CUs x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix


def tri_flop(n: int) -> float:
    """Flops of the Householder reduction of an n x n complex Hermitian matrix to
    real tridiagonal form: (16/3) n^3 real flops (a complex multiply-add is 8)."""
    return 16.0 / 3.0 * n ** 3


def cg_iter_bytes(T: int, P: int, Q: int, M: int) -> float:
    """Algorithmic bytes of one CG iteration: the operator reads p and writes Ap,
    the updates read x, p, r, Ap and write x, r, the p update reads r and writes p
    (10 complex64 volumes), plus one read of the W = M(M+1)/2 penalty masks and
    of the bit-packed sampling mask."""
    V, W = T * P * Q, M * (M + 1) // 2
    return 10 * V * 8 + W * P * Q * 8 + V / 8


def outer_iter_bytes(T: int, P: int, Q: int, M: int, N1: int, N2: int) -> float:
    """Algorithmic bytes of one outer iteration outside the CG: the images (3
    volumes), the lagged sums and their transforms (3 passes over W P Q complex128
    planes), five passes over the s x s complex128 Gram-sized matrices and the
    mask write."""
    V, W, s = T * P * Q, M * (M + 1) // 2, N1 * N2 * M
    return 3 * V * 8 + 3 * W * P * Q * 16 + 5 * s * s * 16 + W * P * Q * 8


def backtr_flop(n: int, nb: int = 64) -> float:
    """Flops of the blocked back-transformation (complex MAC = 8 flop): per block
    of nr reflectors acting on m = n - nb g - 1 rows, V^H V and V T (nr^2 m each),
    then V^H Z and Z - Y W (nr m n each)."""
    tot = 0.0
    for g in range((n - 2) // nb + 1 if n > 1 else 0):
        nr = min(nb, n - 1 - nb * g)
        m = n - nb * g - 1
        tot += 8.0 * (2 * nr * nr * m + 2 * nr * m * n)
    return tot


def tri_launches(n: int) -> int:
    """Launches of one tridiagonalisation (the library's launch schedule): one per
    column up to the last 96, which share one launch."""
    return max(n - 96, 0) + 1


def roofline(kind, avg_ms, T, P, Q, M, N1, N2, nc=0):
    """Roofline entry of one kernel class.  The filter product and the
    back-transformation are FP64 MFMA contractions (the spectral lag sums that
    replace the filter product where the shape allows are FP64 vector work); the
    tridiagonalisation is FP64 vector arithmetic, (16/3) s^3 flops per
    decomposition, reported per launch; every other class is bound by HBM."""
    s = N1 * N2 * M
    if kind == "filter" and spectral_groups(N1, N2, M):  # FP64 vector arithmetic
        flop = spectral_flop(N1, N2, M)
        ach = flop / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "kernel": kind, "achieved": round(ach, 2), "peak": FP64_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP64_VALU_PEAK_TFLOPS, 4), "traffic": None,
                "flop_per_launch": flop, "avg_launch_ms": round(avg_ms, 5)}
    if kind in ("filter", "backtr"):
        flop = 8.0 * s ** 3 if kind == "filter" else backtr_flop(s)
        ach = flop / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": kind, "achieved": round(ach, 2), "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                "flop_per_launch": flop, "avg_launch_ms": round(avg_ms, 5)}
    if kind == "tri":  # FP64 vector work, per launch
        launches = tri_launches(s)
        flop = tri_flop(s) / launches
        ms = avg_ms / launches
        ach = flop / (ms * 1e-3) / 1e12
        return {"bound": "alu", "kernel": kind, "achieved": round(ach, 3), "peak": FP64_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP64_VALU_PEAK_TFLOPS, 4), "traffic": None,
                "flop_per_launch": flop, "launches_per_decomposition": launches,
                "avg_launch_ms": round(ms, 6)}
    nbytes = algorithmic_bytes(kind, T, P, Q, M, N1, N2, nc)
    ach = nbytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kind, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": nbytes,
            "avg_launch_ms": round(avg_ms, 6)}


def kernel_source_hash() -> str:
    """SHA-256 of the kernel sources with comments and blank lines removed, so that
    a counter summary stays attached to the code it measured across comment edits."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_1704_04511_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name)) as f:
            text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
        for line in text.splitlines():
            code = re.sub(r"//.*", "", line).strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_traffic(kind: str):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "c3_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if kernel_source_hash() != rec.get("source_sha256"):
        return None
    return rec.get("bytes_per_launch", {}).get(kind)


def cpu_baseline(pb, n_outer: int = 1):
    """FP64 oracle on a bounded sample: the first outer iteration(s) of the workload.
    Returns the baseline record and the oracle's images after those iterations."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    img = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, n_outer, pb.n_cg, p=pb.p, gamma=pb.gamma,
                      eps0_frac=pb.eps0_frac)
    dt = time.perf_counter() - t0
    return {"value": n_outer / dt, "unit": "IRLS iter/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_outer} of {pb.n_irls} outer iterations ({pb.n_cg} CG each) of the same "
                      f"256x256x20 workload, NumPy/SciPy FP64, {dt:.1f} s wall"}, img


def measure_batch(steps: int, warmup: int, slices: int = 32, oracle_seconds: float = 0.0,
                  check_bits: bool = True, grouping: int = -1) -> dict:
    """Batch of uneven slices (9x9x5, 15 x 10 each) in lock step with shared batched
    eigen-decompositions, against the same slices one plan at a time."""
    import numpy as np
    import torch

    import paper_1704_04511_amd as slrx
    import workload

    torch.cuda.set_device(0)
    slrx.set_cg_grouping(grouping)
    specs = workload.batch_specs(slices, seed=11)
    pbs = [workload.make_problem(name=f"slice{j}", **sp) for j, sp in enumerate(specs)]
    plans = []
    for pb in pbs:
        T, P, Q = pb.b.shape
        pl = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M,
                       slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg))
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        plans.append(pl)
    irls_total = sum(pb.n_irls for pb in pbs)
    for _ in range(warmup):
        slrx.run_batch(plans)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        slrx.run_batch(plans)
    torch.cuda.synchronize()
    dt_batch = (time.perf_counter() - t0) / steps
    out = {"slices": len(plans), "slices_per_s": round(len(plans) / dt_batch, 3),
           "ms_per_batch": round(dt_batch * 1e3, 3), "irls_iters_per_s": round(irls_total / dt_batch, 2)}
    batch_imgs = [pl.images() for pl in plans]
    t0 = time.perf_counter()
    for pl in plans:
        pl.run()
        pl.sync()
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    out["one_at_a_time_slices_per_s"] = round(len(plans) / dt_seq, 3)
    out["batch_speedup"] = round(dt_seq / dt_batch, 3)
    if check_bits:
        seq_imgs = [pl.images() for pl in plans]
        out["batch_equals_single_run_bitwise"] = all(np.array_equal(x, y) for x, y in zip(batch_imgs, seq_imgs))
    # the CG strategy of the engine steps on this draw and on a draw of small slices
    # (32 x 64x64x8, 5x5x3, 15 x 10): per problem, grouped, and the tuner's choice
    def timed_batch(ps, mode, reps=3):
        slrx.set_cg_grouping(mode)
        try:
            slrx.run_batch(ps)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                slrx.run_batch(ps)
            torch.cuda.synchronize()
            return len(ps) * reps / (time.perf_counter() - t)
        finally:
            slrx.set_cg_grouping(grouping)
    small = [workload.make_problem(seed=500 + i, P=64, Q=64, T=8, K=1, R=4, N1=5, N2=5, M=3, n_irls=15, n_cg=10)
             for i in range(32)]
    splans = []
    for pb in small:
        pl = slrx.Plan(64, 64, 8, 5, 5, 3, slrx.make_params(lam=pb.lam, n_irls=15, n_cg=10))
        pl.set_kspace(pb.b)
        pl.set_mask(pb.S)
        splans.append(pl)
    for _ in range(2):  # settle the tuner for the small draw
        slrx.run_batch(splans)
    out["cg_strategy_slices_per_s"] = {
        "this_draw": {"per_problem": round(timed_batch(plans, 0), 2), "grouped": round(timed_batch(plans, 1), 2)},
        "small_slices_32x64x64x8": {"per_problem": round(timed_batch(splans, 0), 2),
                                    "grouped": round(timed_batch(splans, 1), 2),
                                    "tuned": round(timed_batch(splans, -1), 2)},
    }
    for pl in splans:
        pl.close()
    if oracle_seconds > 0:
        import oracle
        # whole slices of the same batch through the oracle until the time is up
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        done = 0
        while done < len(pbs) and time.perf_counter() - t0 < oracle_seconds:
            pb = pbs[done]
            oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg)
            done += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / dt, "unit": "slices/s", "cores": cores, "kind": "oracle",
                               "sample": f"slices 0..{done - 1} of the same batch, whole (all outer "
                                         f"iterations), NumPy/SciPy FP64, {dt:.1f} s wall"}
    for pl in plans:
        pl.close()
    return out


def bench_batch(args) -> int:
    """32 independent slices of uneven sizes: lock-step batch (shared batched
    eigen-decompositions) vs one plan at a time."""
    m = measure_batch(args.steps, args.warmup, 32, 0.0 if args.no_cpu_baseline else 10.0,
                      grouping=args.cg_grouping)
    out = {
        "metric": "slices/s, batch of 32 uneven slices (batched vs one at a time)",
        "value": m["slices_per_s"], "unit": "slices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_batch"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": "32 slices, P=Q in {96,128,160,192,256}, T in {8,12,16,20}, K in {1,2}, "
                               "R in {4,6,8}, filter 9x9x5, 15 IRLS x 10 CG", "slices": m["slices"]},
    }
    out.update({k: v for k, v in m.items() if k not in ("slices", "slices_per_s", "ms_per_batch")})
    print(json.dumps(out))
    return 0


def measure_serve(n: int, rate: float = 50.0, budget: int = 16 << 30, slots: int = 16) -> dict:
    """Poisson request stream: 90% batch-style slices (9x9x5, 15 x 10), 10% at
    256x256x20 with 15x15x5 (20 x 15); latency = completion - submission."""
    import numpy as np
    import torch

    import paper_1704_04511_amd as slrx
    import workload

    torch.cuda.set_device(0)
    rng = np.random.default_rng(7)
    specs = workload.batch_specs(n, seed=7)
    reqs = []
    for j in range(n):
        if rng.random() < 0.1:
            kw = dict(workload.CONFIGS["c3"])
        else:
            kw = dict(specs[j])
        kw["seed"] = 100000 + j
        reqs.append(workload.make_problem(name=f"req{j}", **kw))
    gaps = rng.exponential(1.0 / rate, size=n)
    srv = slrx.Server(budget, max_slots=slots)
    # warm-up: one request of each shape class (plans, engine buffers, code objects)
    warm = [reqs[0]] + [p for p in reqs if p.N1 == 15][:1]
    for pb in warm:
        t = srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M,
                            slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg))
        srv.wait(t)
        srv.release(t)
    torch.cuda.synchronize()
    tickets = []
    peak = 0
    t_next = time.perf_counter()
    for pb, g in zip(reqs, gaps):
        t_next += g
        while time.perf_counter() < t_next:
            time.sleep(0.0005)
        tickets.append(srv.submit_data(pb.b, pb.S, pb.N1, pb.N2, pb.M,
                                       slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg)))
        peak = max(peak, srv.usage()[0])
    for t in tickets:
        srv.wait(t)
    infos = [srv.info(t) for t in tickets]
    srv.close()
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
    span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
    return {"requests": n, "solves_per_s": round(len(infos) / span, 3),
            "latency_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "latency_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "latency_mean_ms": round(float(lat.mean()) * 1e3, 2),
            "arrival_rate_per_s": rate, "budget_bytes": budget, "max_slots": slots,
            "peak_server_bytes_at_submissions": int(peak),
            "large_requests": int(sum(1 for p in reqs if p.N1 == 15))}


def bench_serve(args) -> int:
    """Poisson request stream (mean 50/s): 90% batch-style slices, 10% 256x256x20 with 15x15x5."""
    m = measure_serve(args.requests)
    out = {
        "metric": "p50/p99 reconstruction latency and solves/s, Poisson stream at 50/s",
        "value": m["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": m["requests"],
        "warmup": 2, "ms_per_step": round(1e3 / m["solves_per_s"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": f"{m['requests']} requests, exponential gaps mean 20 ms (seed 7); 90% "
                               "batch-style slices (9x9x5, 15x10), 10% 256x256x20 (15x15x5, 20x15)",
                   "max_slots": m["max_slots"], "budget_bytes": m["budget_bytes"]},
    }
    out.update({k: v for k, v in m.items() if k not in ("solves_per_s",)})
    print(json.dumps(out))
    return 0


def t2_map(img, te_ms, mask):
    """Mono-exponential T2 per pixel: least-squares line through log|rho_t| against TE."""
    import numpy as np
    y = np.log(np.maximum(np.abs(img[:, mask]), 1e-30))  # [T][pixels]
    t = np.asarray(te_ms, dtype=np.float64)
    tc = t - t.mean()
    slope = (tc[:, None] * (y - y.mean(axis=0))).sum(axis=0) / (tc * tc).sum()
    with np.errstate(divide="ignore"):
        return -1.0 / slope


def bench_c2(args) -> int:
    """128x128x16 (filter 9x9x5, 15 x 10): IRLS iterations/s, NRMSE against the oracle, and
    mono-exponential T2 maps fitted the same way to the GPU result, the oracle and the truth."""
    import numpy as np
    import torch

    import oracle
    import paper_1704_04511_amd as slrx
    import workload

    torch.cuda.set_device(0)
    pb = workload.config_problem("c2")
    T, P, Q = pb.b.shape
    prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p, gamma=pb.gamma,
                           eps0_frac=pb.eps0_frac)
    plan = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm)
    plan.set_kspace(pb.b)
    plan.set_mask(pb.S)
    for _ in range(args.warmup):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    img = plan.images()
    te = 10.0 * (np.arange(T) + 1)
    torch.cuda.synchronize()
    tf = time.perf_counter()
    t2_dev, _ = plan.fit_t2(te)  # per-pixel fit on the GPU (host copy of the maps included)
    fit_ms = (time.perf_counter() - tf) * 1e3
    plan.close()
    # the GIRAF approximation on the same data (circular along the echoes too; Sec. IV, Fig. 3)
    gprm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p, gamma=pb.gamma,
                            eps0_frac=pb.eps0_frac, giraf=True)
    with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, gprm) as gp:
        gp.set_kspace(pb.b)
        gp.set_mask(pb.S)
        gp.run()
        gp.sync()
        img_giraf = gp.images()
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ora = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, p=pb.p, gamma=pb.gamma,
                      eps0_frac=pb.eps0_frac)
    dto = time.perf_counter() - t0
    mask = np.abs(pb.truth[0]) > 0.1 * np.abs(pb.truth[0]).max()
    t2g, t2o, t2t, t2f = (t2_map(v, te, mask) for v in (img, ora, pb.truth, img_giraf))
    nrm = lambda a: float(np.linalg.norm(a - pb.truth) / np.linalg.norm(pb.truth))
    rel = lambda a, b: float(np.median(np.abs(a - b) / np.abs(b)))
    out = {
        "metric": "IRLS iters/s (128x128x16, filter 9x9x5)", "value": round(pb.n_irls * args.steps / dt, 3),
        "unit": "IRLS iter/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": "128x128 x 16 echoes, K=2, R=6, filter 9x9x5 (s=405), 15 IRLS x 10 CG",
                   "n_irls": pb.n_irls, "n_cg": pb.n_cg},
        "nrmse_vs_oracle": float(f"{np.linalg.norm(img - ora) / np.linalg.norm(ora):.3e}"),
        "t2_pixels": int(mask.sum()),
        "t2_median_rel_err_gpu_vs_truth": round(rel(t2g, t2t), 5),
        "t2_median_rel_err_oracle_vs_truth": round(rel(t2o, t2t), 5),
        "t2_median_rel_diff_gpu_vs_oracle": float(f"{rel(t2g, t2o):.3e}"),
        "t2_gpu_fit_max_rel_diff_vs_host_fit": float(f"{np.max(np.abs(t2_dev[mask] - t2g) / np.abs(t2g)):.3e}"),
        "t2_gpu_fit_ms": round(fit_ms, 3),
        "approximation_study": {"recon_nrmse_vs_truth_hybrid": round(nrm(img), 5),
                                "recon_nrmse_vs_truth_giraf": round(nrm(img_giraf), 5),
                                "t2_median_rel_err_vs_truth_hybrid": round(rel(t2g, t2t), 5),
                                "t2_median_rel_err_vs_truth_giraf": round(rel(t2f, t2t), 5)},
        "cpu_baseline": {"value": pb.n_irls / dto, "unit": "IRLS iter/s", "cores": cores, "kind": "oracle",
                         "sample": f"the whole reconstruction ({pb.n_irls} outer iterations), {dto:.1f} s wall"},
    }
    print(json.dumps(out))
    return 0


def bench_mc(args) -> int:
    """Multichannel workload (128x128 x 12 echoes, 12 coils, R=8, filter 9x9x5, 15 x 10):
    IRLS iterations/s, the per-class breakdown and rooflines, NRMSE against the FP64
    oracle and the oracle's own time for the whole reconstruction."""
    import numpy as np
    import torch

    import oracle
    import paper_1704_04511_amd as slrx
    import workload

    torch.cuda.set_device(0)
    pb = workload.config_problem("mc")
    nc, T, P, Q = pb.b.shape
    mk = lambda kt, classes=None: slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p,
                                                    gamma=pb.gamma, eps0_frac=pb.eps0_frac, ktime=kt,
                                                    ktime_classes=classes)
    plan = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, mk(False))
    plan.set_mask(pb.S)
    plan.set_coils(pb.coils, pb.b)
    for _ in range(args.warmup):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    img = plan.images()
    plan.set_params(mk(True))  # one more reconstruction with every class timed
    plan.run()
    plan.sync()
    st = plan.stats()
    plan.close()
    kms, kcnt = st["kernel_ms"], st["kernel_count"]
    own = [k for k in ("rows", "coil", "cols", "fin", "update", "gram", "tri", "backtr", "filter", "masks")
           if kcnt[k] > 0]
    roofs = {k: roofline(k, kms[k] / kcnt[k], T, P, Q, pb.M, pb.N1, pb.N2, nc) for k in own}
    dom = max(own, key=lambda k: kms[k])
    out = {
        "metric": "IRLS iters/s (128x128x12, 12 coils, filter 9x9x5)",
        "value": round(pb.n_irls * args.steps / dt, 3), "unit": "IRLS iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": "128x128 x 12 echoes, 12 coils (Sec. II.A multichannel model), K=2, R=8, "
                               "filter 9x9x5 (s=405), 15 IRLS x 10 CG", "ncoils": nc,
                   "n_irls": pb.n_irls, "n_cg": pb.n_cg},
        "roofline": roofs[dom],
        "roofline_by_kernel": {k: {kk: v for kk, v in r.items() if kk in ("bound", "achieved", "unit", "frac")}
                               for k, r in roofs.items()},
        "phases_ms_per_step": {k: round(kms[k], 3) for k in kms if kcnt[k] > 0},
        "recon_nrmse_vs_truth": round(float(np.linalg.norm(img - pb.truth) / np.linalg.norm(pb.truth)), 5),
    }
    if not args.no_cpu_baseline:
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        ora = oracle.irls(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, p=pb.p, gamma=pb.gamma,
                          eps0_frac=pb.eps0_frac, coils=pb.coils)
        dto = time.perf_counter() - t0
        out["nrmse_vs_oracle"] = float(f"{np.linalg.norm(img - ora) / np.linalg.norm(ora):.3e}")
        out["cpu_baseline"] = {"value": pb.n_irls / dto, "unit": "IRLS iter/s", "cores": cores, "kind": "oracle",
                               "sample": f"the whole reconstruction ({pb.n_irls} outer iterations), {dto:.1f} s wall"}
    print(json.dumps(out))
    return 0


def bench_hlr(args) -> int:
    """The 256x256x20 data under the pixel-wise prior (HLR-Voxel, 1x1x5 filter per
    pixel, 20 x 15): IRLS iterations/s, the per-class breakdown, NRMSE against the
    FP64 oracle on the first outer iterations, and the oracle's time for them."""
    import numpy as np
    import torch

    import oracle
    import paper_1704_04511_amd as slrx
    import workload

    torch.cuda.set_device(0)
    pb = workload.config_problem("hlr")
    T, P, Q = pb.b.shape
    mk = lambda kt, n_irls=pb.n_irls: slrx.make_params(lam=pb.lam, n_irls=n_irls, n_cg=pb.n_cg, p=pb.p,
                                                        gamma=pb.gamma, eps0_frac=pb.eps0_frac, ktime=kt,
                                                        voxel=True)
    plan = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, mk(False))
    plan.set_kspace(pb.b)
    plan.set_mask(pb.S)
    for _ in range(args.warmup):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    img = plan.images()
    plan.set_params(mk(True))  # one more reconstruction with every class timed
    plan.run()
    plan.sync()
    st = plan.stats()
    kms, kcnt = st["kernel_ms"], st["kernel_count"]
    own = [k for k in ("rows", "cols", "fin", "update", "voxel") if kcnt[k] > 0]
    roofs = {k: roofline(k, kms[k] / kcnt[k], T, P, Q, pb.M, pb.N1, pb.N2) for k in own}
    dom = max(own, key=lambda k: kms[k])
    out = {
        "metric": "IRLS iters/s (256x256x20, HLR-Voxel 1x1x5 per pixel)",
        "value": round(pb.n_irls * args.steps / dt, 3), "unit": "IRLS iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": "the 256x256 x 20-echo T2 series (K=2, smooth phase, R=8) under the pixel-wise "
                               "Hankel prior (Sec. II.E): 65536 per-pixel 5x5 Gram eigen-decompositions per "
                               "outer iteration, 20 IRLS x 15 CG", "n_irls": pb.n_irls, "n_cg": pb.n_cg},
        "roofline": roofs[dom],
        "roofline_by_kernel": {k: {kk: v for kk, v in r.items() if kk in ("bound", "achieved", "unit", "frac")}
                               for k, r in roofs.items()},
        "phases_ms_per_step": {k: round(kms[k], 3) for k in kms if kcnt[k] > 0},
        "voxel_weight_update_ms": round(kms["voxel"] / max(kcnt["voxel"], 1), 4),
        "recon_nrmse_vs_truth": round(float(np.linalg.norm(img - pb.truth) / np.linalg.norm(pb.truth)), 5),
    }
    if not args.no_cpu_baseline:
        n_out = 2
        plan.set_params(mk(False, n_out))
        plan.run()
        plan.sync()
        part = plan.images()
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        ora = oracle.irls_voxel(pb.b, pb.S, pb.M, pb.lam, n_out, pb.n_cg, p=pb.p, gamma=pb.gamma,
                                eps0_frac=pb.eps0_frac)
        dto = time.perf_counter() - t0
        out["nrmse_vs_oracle_first_outer"] = float(f"{np.linalg.norm(part - ora) / np.linalg.norm(ora):.3e}")
        out["cpu_baseline"] = {"value": n_out / dto, "unit": "IRLS iter/s", "cores": cores, "kind": "oracle",
                               "sample": f"the first {n_out} outer iterations of the same workload, {dto:.1f} s wall"}
    plan.close()
    print(json.dumps(out))
    return 0


def bench_direct(args) -> int:
    """The approximation study of Sec. IV / Fig. 2 on synthetic data: the proposed
    method (FFT-based, hybrid lifting) against IRLS-direct (explicit linear lifting,
    no approximations) on the same problem at the same iteration counts, both on
    the GPU: time to solution, the speed-up, and how close the two solutions are.
    Data: the 64x64x8 (5x5x3, 15 x 10) workload, checked against the FP64 oracle,
    and the 128x128x16 one (9x9x5, s = 405, 15 x 10; GPU only)."""
    import numpy as np
    import torch

    import oracle
    import paper_1704_04511_amd as slrx
    import workload

    torch.cuda.set_device(0)

    def timed(pb, direct):
        T, P, Q = pb.b.shape
        prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p, gamma=pb.gamma,
                               eps0_frac=pb.eps0_frac, direct=direct)
        with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            for _ in range(args.warmup):
                pl.run()
                pl.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                pl.run()
                pl.sync()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / args.steps, pl.images()

    nr = lambda a, b: float(f"{np.linalg.norm(a - b) / np.linalg.norm(b):.4e}")

    def direct_roofline(pb):
        """IRLS-direct on the 128x128x16 data with its two classes timed: the Gram
        matrix (lifting + zgemm, 8 s^2 rows flop on FP64 MFMA) and the CG (per operator
        application lifting + cgemm, 8 s^2 rows flop on FP32 MFMA, + adjoint)."""
        T, P, Q = pb.b.shape
        s = pb.N1 * pb.N2 * pb.M
        nrows = (T - pb.M + 1) * (P - pb.N1 + 1) * (Q - pb.N2 + 1)
        prm = slrx.make_params(lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p, gamma=pb.gamma,
                               eps0_frac=pb.eps0_frac, direct=True, ktime=True, ktime_classes=("gram", "direct"))
        with slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, prm) as pl:
            pl.set_kspace(pb.b)
            pl.set_mask(pb.S)
            pl.run()
            pl.sync()
            st = pl.stats()
        kms, kcnt = st["kernel_ms"], st["kernel_count"]
        gram_ms = kms["gram"] / kcnt["gram"]
        cg_ms = kms["direct"] / kcnt["direct"]
        gram_tf = 8.0 * s * s * nrows / (gram_ms * 1e-3) / 1e12
        cg_tf = (pb.n_cg + 1) * 8.0 * s * s * nrows / (cg_ms * 1e-3) / 1e12
        return {
            "gram": {"bound": "mfma", "achieved": round(gram_tf, 2), "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(gram_tf / FP64_MFMA_PEAK_TFLOPS, 4),
                     "ms_per_outer_iteration": round(gram_ms, 3), "flop": 8.0 * s * s * nrows},
            "cg": {"bound": "mfma", "achieved": round(cg_tf, 2), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(cg_tf / FP32_MFMA_PEAK_TFLOPS, 4), "ms_per_least_squares_step": round(cg_ms, 3),
                   "flop": (pb.n_cg + 1) * 8.0 * s * s * nrows,
                   "note": "the GEMM flops of the n_cg + 1 operator applications over the whole CG region "
                           "(lifting and adjoint gathers included in the time)"},
        }

    rows = {}
    for name in ("c1", "c2"):
        pb = workload.config_problem(name)
        t_prop, x_prop = timed(pb, False)
        t_dir, x_dir = timed(pb, True)
        rows[name] = {"shape": list(pb.b.shape), "filter": [pb.N1, pb.N2, pb.M], "n_irls": pb.n_irls,
                      "n_cg": pb.n_cg, "proposed_ms": round(t_prop * 1e3, 3), "direct_ms": round(t_dir * 1e3, 3),
                      "speedup": round(t_dir / t_prop, 2), "proposed_nrmse_vs_truth": nr(x_prop, pb.truth),
                      "direct_nrmse_vs_truth": nr(x_dir, pb.truth), "proposed_vs_direct": nr(x_prop, x_dir)}
    out = {
        "metric": "speed-up of the proposed FFT-based IRLS over IRLS-direct (64x64x8, 5x5x3)",
        "value": rows["c1"]["speedup"], "unit": "x", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rows["c1"]["direct_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": "the 64x64x8 T2 series (K=1, R=4, 5x5x3 filter, 15 x 10) and the 128x128x16 one "
                               "(K=2, R=6, 9x9x5, 15 x 10): proposed (hybrid circular lifting, FFT-based steps) "
                               "vs IRLS-direct (explicit linear lifting, GEMM-based steps)"},
        "by_workload": rows,
        "note": "the paper reports 7.5x for its MATLAB implementations on real data (Fig. 2); here both methods "
                "run on one MI355X",
    }
    out["roofline_direct_128x128x16"] = direct_roofline(workload.config_problem("c2"))
    out["roofline"] = dict(out["roofline_direct_128x128x16"]["cg"], kernel="direct CG (lifting, cgemm, adjoint)")
    if not args.no_cpu_baseline:
        pb = workload.config_problem("c1")
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        ora = oracle.irls_direct(pb.b, pb.S, pb.N1, pb.N2, pb.M, pb.lam, pb.n_irls, pb.n_cg, p=pb.p, gamma=pb.gamma,
                                 eps0_frac=pb.eps0_frac)
        dto = time.perf_counter() - t0
        _, x_dir = timed(pb, True)
        out["direct_nrmse_vs_oracle"] = nr(x_dir, ora)
        out["cpu_baseline"] = {"value": round(dto * 1e3, 1), "unit": "ms per IRLS-direct reconstruction",
                               "cores": cores, "kind": "oracle",
                               "sample": f"the whole 64x64x8 IRLS-direct reconstruction, {dto:.1f} s wall"}
    print(json.dumps(out))
    return 0


def bench_calib(args) -> int:
    """Plain device-to-device copy of a known size (--calib-mb MiB read and written
    per launch), to calibrate rocprofv3 FETCH_SIZE / WRITE_SIZE against bytes."""
    import torch
    n = args.calib_mb * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        print(json.dumps({"copy_mib": args.calib_mb, "ms": round(ms, 4),
                          "gbs_read_plus_write": round(2 * args.calib_mb * (1 << 20) / ms / 1e6, 1)}), flush=True)
    return 0


# Kernel classes of the bench's rooflines -> the kernel names they cover and the kernel
# whose dispatch count defines "one launch" (None: one launch = one decomposition,
# counted by the tridiagonalisation's single-workgroup tail).
PROFILE_CLASSES = {
    "rows": (("k_rows_t",), "k_rows_t"),
    "cols": (("k_cols_pen",), "k_cols_pen"),
    "fin": (("k_rows_fin",), "k_rows_fin"),
    "update": (("k_update",), "k_update"),
    "gram": (("k_gram_",), "k_gram_assemble"),
    "tri": (("k_tri_",), "k_tri_col"),
    "tdeig": (("k_dc_",), None),
    "backtr": (("k_bt_",), None),
    "filter": (("k_spec_", "k_eps", "k_weights", "k_filter_product"), None),
    "masks": (("k_mask_", "k_diagsum"), None),
}


def _kernel_short(name: str) -> str:
    import re
    name = re.sub(r"^void ", "", name)
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _csv_rows(root: str, sub: str, suffix: str):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(root, sub, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {os.path.join(root, sub)}")
    rows = []
    for fn in files:
        with open(fn, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _counter_per_kernel(root: str, sub: str):
    """{kernel: [dispatches, summed counter KiB]} from a rocprofv3 --pmc csv run."""
    agg = {}
    for r in _csv_rows(root, sub, "counter_collection.csv"):
        k = _kernel_short(r["Kernel_Name"])
        a = agg.setdefault(k, [0, 0.0])
        a[0] += 1
        a[1] += float(r["Counter_Value"])
    return agg


def grouped_rooflines(root: str, sub: str) -> list:
    """HBM rooflines of the grouped CG kernels of the 32-slice draw: the algorithmic
    bytes of one grouped launch (the sum over the slices of each pass's bytes per
    launch) over the average duration of that kernel's dispatches with the largest
    grid (the launches that hold the whole draw; the smaller-slice draw of the
    strategy comparison launches smaller grids)."""
    import workload
    specs = workload.batch_specs(32, seed=11)
    V = sum(sp["T"] * sp["P"] * sp["Q"] for sp in specs)
    PQ = sum(sp["P"] * sp["Q"] for sp in specs)
    W = 15  # M = 5 for every slice of the draw
    nbytes = {"k_group_rows": 32 * V, "k_group_pen<5>": 16 * V + 8 * W * PQ, "k_group_fin": 25 * V,
              "k_group_update": 48 * V}
    rows = _csv_rows(root, sub, "group_dispatches.csv")
    gcols = [c for c in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z") if c in rows[0]] or ["Grid_Size"]
    by = {}
    for r in rows:
        name = _kernel_short(r["Kernel_Name"]).split("::")[-1]
        key = next((k for k in nbytes if name.startswith(k)), None)
        if key is None:
            continue
        grid = 1
        for c in gcols:
            grid *= int(r[c])
        by.setdefault(key, []).append((grid, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = ["", f"# grouped CG launches of the whole draw (sum of T*P*Q = {V} elements, {V * 8 / 1e6:.0f} MB per "
               "complex FP32 vector: the working set is beyond the 256 MB MALL) against the 8 TB/s HBM peak: "
               "algorithmic bytes per launch / average duration of the launches with the largest grid "
               "(rows: the p-update launches' 32 B per element; the one initial-residual launch per outer "
               "iteration moves 16 and is averaged in)",
           f"{'kernel':<16} {'launches':>9} {'MB_per_launch':>14} {'avg_us':>9} {'GB_per_s':>10} {'frac_of_8TB':>12}"]
    for key, d in by.items():
        gmax = max(g for g, _ in d)
        ns = [t for g, t in d if g == gmax]
        us = sum(ns) / len(ns) * 1e-3
        gbs = nbytes[key] / (us * 1e-6) / 1e9
        out.append(f"{key:<16} {len(ns):>9} {nbytes[key] / 1e6:>14.1f} {us:>9.1f} {gbs:>10.1f} "
                   f"{gbs / 8000:>12.3f}")
    return out


def summarize_profiles(args) -> int:
    """Write profiles/c3_kernel_trace.txt, c3_hbm_counters.txt and c3_traffic.json from
    the rocprofv3 csv output of the runs named in their headers (no GPU needed)."""
    root = args.prof_root
    prof = os.path.join(ROOT, "profiles")
    pre = "cd /tmp && export TMPDIR=/tmp && cd /root/repo && "
    # the c3 runs share one tuner cache: an unprofiled run of the same command
    # settles and records the launch choices first (a profiler changes the timings
    # they are made from), and every profiled run reads them back
    pre_c3 = pre + "export SLRX_TUNE_CACHE=gpurun_out/tune_c3.txt && "
    c3 = "python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-extras"
    c3_pmc = "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-extras --n-irls 2"
    calib = "python3 bench.py --workload calib --calib-mb 256"
    # kernel traces: (folder, file, what, command)
    traces = [
        ("prof_c3", "c3_kernel_trace.txt", "256x256x20 workload (filter 15x15x5, s=1125; 20 outer x 15 CG): 1 "
         "warm-up, 1 timed and 1 fully instrumented reconstruction (divide totals by 3 per reconstruction)", c3),
        ("prof_hlr", "hlr_kernel_trace.txt", "256x256x20 data under HLR-Voxel (1x1x5 per pixel; 20 outer x 15 "
         "CG): 1 warm-up, 1 timed and 1 fully instrumented reconstruction (divide totals by 3)",
         "python3 bench.py --workload hlr --steps 1 --warmup 1 --no-cpu-baseline"),
        ("prof_direct", "direct_kernel_trace.txt", "proposed vs IRLS-direct on the 64x64x8 (5x5x3) and "
         "128x128x16 (9x9x5) workloads, 15 x 10 each: per workload and method 1 warm-up and 1 timed "
         "reconstruction", "python3 bench.py --workload direct --steps 1 --warmup 1 --no-cpu-baseline"),
    ]
    traces.append(("prof_batch_grouped", "batch_grouped_kernel_trace.txt",
                   "the 32-slice batch draw (96..256 squared, 8..20 echoes, 9x9x5, 15 x 10) with the CG in "
                   "grouped launches: 1 warm-up and 1 timed batch, then the single-plan runs and the strategy "
                   "comparisons of the batch line", "python3 bench.py --workload batch --steps 1 --warmup 1 "
                   "--no-cpu-baseline --cg-grouping 1"))
    for sub, fname, what, cmd in traces:
        if not os.path.isdir(os.path.join(root, sub)):
            continue
        st = _csv_rows(root, sub, "kernel_stats.csv")
        tot = sum(float(r["TotalDurationNs"]) for r in st)
        lines = [f"# Kernel trace, {what}"]
        if sub == "prof_c3":
            lines.append("# the tuner's launch choices read from that cache, recorded first by the same command "
                         "without the profiler")
        lines += [
                  f"# command: {pre_c3 if sub == 'prof_c3' else pre}rocprofv3 --kernel-trace --stats -f csv "
                  f"-d gpurun_out/{sub} -o run -- {cmd}",
                  "# durations from the kernel trace (rocprofv3 kernel_stats)",
                  f"{'kernel':<72} {'calls':>8} {'total_ms':>10} {'avg_us':>9} {'pct':>6}"]
        for r in sorted(st, key=lambda r: -float(r["TotalDurationNs"])):
            ms = float(r["TotalDurationNs"]) * 1e-6
            lines.append(f"{_kernel_short(r['Name'])[:72]:<72} {int(r['Calls']):>8} {ms:>10.3f} "
                         f"{float(r['AverageNs']) * 1e-3:>9.2f} {100 * ms * 1e6 / tot:>6.2f}")
        if sub == "prof_batch_grouped":
            lines += grouped_rooflines(root, sub)
        with open(os.path.join(prof, fname), "w") as f:
            f.write("\n".join(lines) + "\n")
    # counters, calibrated by the copy; stamped with the hash of the kernel sources
    # that the counter runs profiled (written on the GPU side before those runs)
    hfile = os.path.join(root, "pmc_source_sha256.txt")
    if not os.path.isfile(hfile):
        print(json.dumps({"written": "kernel traces only", "note": f"{hfile} missing: counters not summarised"}))
        return 0
    with open(hfile) as f:
        profiled_hash = f.read().strip()
    fetch = _counter_per_kernel(root, "pmc_fetch")
    write = _counter_per_kernel(root, "pmc_write")
    cf = _counter_per_kernel(root, "pmc_copy_fetch")
    cw = _counter_per_kernel(root, "pmc_copy_write")
    copy_k = max(cf, key=lambda k: cf[k][1] / cf[k][0])  # the copy reads; the buffer fill before it does not
    kib = args.calib_mb * 1024.0
    f_copy, w_copy = cf[copy_k][1] / cf[copy_k][0], cw[copy_k][1] / cw[copy_k][0]
    sf, sw = kib / f_copy, kib / w_copy
    lines = ["# HBM traffic per dispatch, 256x256x20 workload (filter 15x15x5), two outer iterations",
             "# commands (each its own run):",
             f"#   {pre_c3}rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_fetch -o run -- {c3_pmc}",
             f"#   {pre_c3}rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_write -o run -- {c3_pmc}",
             "# (the tuner's launch choices read from that cache, recorded by an unprofiled run of the "
             "command of c3_kernel_trace.txt)",
             f"# calibration: a {args.calib_mb} MiB device copy ({copy_k}) under the same counters:",
             f"#   {pre}rocprofv3 --pmc FETCH_SIZE -f csv -d gpurun_out/pmc_copy_fetch -o run -- {calib}",
             f"#   {pre}rocprofv3 --pmc WRITE_SIZE -f csv -d gpurun_out/pmc_copy_write -o run -- {calib}",
             f"# copy: FETCH_SIZE {f_copy:.1f} KiB, WRITE_SIZE {w_copy:.1f} KiB for {kib:.0f} KiB moved each way "
             f"-> scale fetch x{sf:.3f}, write x{sw:.3f}",
             f"# summaries written by: python3 bench.py --workload profiles --prof-root gpurun_out",
             f"{'kernel':<52} {'n':>6} {'fetch_KiB':>11} {'write_KiB':>11} {'scaled_MB':>10}"]
    per = {}
    for k in fetch:
        n = fetch[k][0]
        fk = fetch[k][1] / n
        wk = write.get(k, [n, 0.0])[1] / max(write.get(k, [n, 0.0])[0], 1)
        per[k] = (n, fk, wk, (fk * sf + wk * sw) * 1024.0)
    for k, (n, fk, wk, b) in sorted(per.items(), key=lambda kv: -kv[1][0] * kv[1][3]):
        lines.append(f"{k[:52]:<52} {n:>6} {fk:>11.1f} {wk:>11.1f} {b / 1e6:>10.3f}")
    with open(os.path.join(prof, "c3_hbm_counters.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    ndec = sum(v[0] for k, v in per.items() if k.startswith("slrx::k_tri_tail") or k.startswith("k_tri_tail"))
    bpl = {}
    for cls, (prefixes, main) in PROFILE_CLASSES.items():
        names = [k for k in per if any(k.split("::")[-1].startswith(p) for p in prefixes)]
        total = sum(per[k][0] * per[k][3] for k in names)
        if main is None:
            units = ndec
        else:
            units = sum(per[k][0] for k in names if k.split("::")[-1].startswith(main))
        if names and units:
            bpl[cls] = total / units
    rec = {"source_sha256": profiled_hash, "workload": "256x256x20 filter 15x15x5",
           "scale_fetch": sf, "scale_write": sw, "bytes_per_launch": bpl}
    with open(os.path.join(prof, "c3_traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps({"written": sorted(os.listdir(prof)), "bytes_per_launch": bpl}))
    return 0


def copy_bandwidth_gbs() -> float:
    """Device-to-device copy of 1 GiB (read + write counted), best of 5, torch's copy kernel."""
    import torch
    n = 1 << 27  # doubles
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    best = 1e9
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return round(2.0 * n * 8 / (best * 1e-3) / 1e9, 1)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-outer", type=int, default=3, help="outer iterations in the CPU oracle sample")
    ap.add_argument("--n-irls", type=int, default=None,
                    help="override the outer iteration count (profiling runs only; changes the workload)")
    ap.add_argument("--workload", choices=("c3", "c2", "mc", "hlr", "direct", "batch", "serve", "calib",
                                           "profiles"),
                    default="c3",
                    help="c3: the 256x256x20 headline line (default); c2: 128x128x16 with T2 maps; "
                         "mc: 12-coil 128x128x12; hlr: the 256x256x20 data under HLR-Voxel; direct: "
                         "proposed vs IRLS-direct; batch: 32 uneven slices; serve: Poisson request stream; "
                         "calib: the plain copy that calibrates the HBM counters")
    ap.add_argument("--requests", type=int, default=120, help="serve: number of requests")
    ap.add_argument("--calib-mb", type=int, default=256, help="calib: MiB copied per launch")
    ap.add_argument("--cg-grouping", type=int, default=-1, choices=(-1, 0, 1),
                    help="batch: CG strategy of the engine steps (-1 tuned, 0 per problem, 1 grouped launches)")
    ap.add_argument("--prof-root", default="gpurun_out",
                    help="profiles: folder holding the rocprofv3 csv output of the runs the summaries name")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the serving and batch measurements (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the library runs each problem on a single device and its "
                                   "multi-GPU sharding is a design, not code; --gpus must be 1",
                          "gpus_requested": args.gpus}))
        return 2
    if args.workload == "profiles":
        return summarize_profiles(args)
    if args.workload == "calib":
        return bench_calib(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "hlr":
        return bench_hlr(args)
    if args.workload == "direct":
        return bench_direct(args)
    if args.workload == "mc":
        return bench_mc(args)
    if args.workload == "c2":
        return bench_c2(args)
    if args.workload == "serve":
        return bench_serve(args)

    import numpy as np
    import torch

    import paper_1704_04511_amd as slrx
    import workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    copy_gbs = copy_bandwidth_gbs()
    pb = workload.config_problem("c3")
    if args.n_irls is not None:
        pb.n_irls = args.n_irls
    T, P, Q = pb.b.shape
    s = pb.N1 * pb.N2 * pb.M
    # Timed region: events around the once-per-iteration stages only (the CG
    # classes would add four event pairs per CG iteration to the stream), plus the
    # phase events of every outer iteration (four per iteration).
    timed_classes = ("gram", "tri", "tdeig", "backtr", "filter", "masks")
    mk = lambda classes, timing=False: slrx.make_params(
        lam=pb.lam, n_irls=pb.n_irls, n_cg=pb.n_cg, p=pb.p, gamma=pb.gamma, eps0_frac=pb.eps0_frac, ktime=True,
        ktime_classes=classes, timing=timing)
    plan = slrx.Plan(P, Q, T, pb.N1, pb.N2, pb.M, mk(timed_classes, True))
    plan.set_kspace(pb.b)
    plan.set_mask(pb.S)
    for _ in range(args.warmup):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
        plan.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = plan.stats()
    img = plan.images()
    ms_step = dt / args.steps * 1e3
    value = pb.n_irls * args.steps / dt
    # one more (untimed) reconstruction with every class timed, for the per-class breakdown
    plan.set_params(mk(None))
    plan.run()
    plan.sync()
    st_all = plan.stats()

    kms, kcnt = st_all["kernel_ms"], st_all["kernel_count"]
    own = [k for k in ("rows", "cols", "fin", "update", "gram", "tri", "tdeig", "backtr", "filter", "masks")
           if kcnt[k] > 0]
    dom = max(own, key=lambda k: kms[k])
    roofs = {k: roofline(k, kms[k] / kcnt[k], T, P, Q, pb.M, pb.N1, pb.N2) for k in own if k != "tdeig"}
    if st["kernel_count"].get(dom, 0) > 0 and dom in roofs:  # the dominant kernel from the timed region itself
        roofs[dom] = roofline(dom, st["kernel_ms"][dom] / st["kernel_count"][dom], T, P, Q, pb.M, pb.N1, pb.N2)
    for k in roofs:
        roofs[k]["traffic"] = measured_traffic(k)
    # the CG iteration against HBM on the method's own bytes: phase time of the CG
    # steps in the timed region (one event pair per outer iteration)
    n_cg_total = pb.n_irls * pb.n_cg
    b_cg = cg_iter_bytes(T, P, Q, pb.M)
    cg_ms = st["ms_cg"] / max(n_cg_total, 1)
    cg_gbs = b_cg / (cg_ms * 1e-3) / 1e9 if cg_ms > 0 else None
    b_outer = outer_iter_bytes(T, P, Q, pb.M, pb.N1, pb.N2)
    b_recon = pb.n_irls * (pb.n_cg * b_cg + b_outer)
    recon_gbs = b_recon / (ms_step * 1e-3) / 1e9
    eig_ms = sum(kms[k] for k in ("tri", "tdeig", "backtr"))
    out = {
        "metric": "IRLS iters/s (256x256x20, FP32 data path / FP64 Gram+eigh)",
        "value": round(value, 3),
        "unit": "IRLS iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64",
        "data": "synthetic",
        "config": {"workload": "T2 series 256x256 x 20 echoes, K=2 exponentials + smooth phase, R=8 "
                               "variable-density masks, filter 15x15x5 (s=1125), 20 IRLS x 15 CG, "
                               "lambda=1e-3, p=0.6",
                   "P": P, "Q": Q, "T": T, "filter": [pb.N1, pb.N2, pb.M], "n_irls": pb.n_irls,
                   "n_cg": pb.n_cg, "parallelism": "single GPU"},
        "roofline": dict(roofs[dom]) if dom in roofs else None,
        "roofline_cg_iteration": {
            "bound": "hbm", "achieved": round(cg_gbs, 1) if cg_gbs else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(cg_gbs / HBM_PEAK_GBS, 4) if cg_gbs else None, "bytes_per_iteration": b_cg,
            "ms_per_iteration": round(cg_ms, 5), "measured_copy_gbs": copy_gbs,
            "note": "algorithmic bytes of one CG iteration (10 volumes, the masks, the bit-packed sampling mask) "
                    "over the CG phase time of the timed region per iteration"},
        "roofline_whole_reconstruction": {
            "bound": "hbm", "achieved": round(recon_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(recon_gbs / HBM_PEAK_GBS, 4), "bytes_per_reconstruction": b_recon,
            "note": "the method's algorithmic bytes per reconstruction over ms_per_step; the eigen-"
                    "decomposition is latency/ALU bound and carries almost none of them"},
        "roofline_by_kernel": {k: {kk: v for kk, v in r.items() if kk in ("bound", "achieved", "unit", "frac")}
                               for k, r in roofs.items()},
        "eigendecomposition": {"ms_per_decomposition": round(eig_ms / pb.n_irls, 4), "s": s,
                               "tri_ms": round(kms["tri"] / pb.n_irls, 4),
                               "tdeig_ms": round(kms["tdeig"] / pb.n_irls, 4),
                               "backtr_ms": round(kms["backtr"] / pb.n_irls, 4),
                               "tri_tflops": round(tri_flop(s) / (kms["tri"] / pb.n_irls * 1e-3) / 1e12, 3)
                               if kms["tri"] > 0 else None},
        "phases_ms_per_step": {k: round(kms[k], 3) for k in kms},
        "phases_note": "per-class times from one extra reconstruction with every class timed",
        "launches_per_step": {k: kcnt[k] for k in kcnt},
        "recon_nrmse_vs_truth": round(float(np.linalg.norm(img - pb.truth) / np.linalg.norm(pb.truth)), 5),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], ora = cpu_baseline(pb, args.cpu_outer)
        # the same number of outer iterations on the GPU, compared with the oracle's images
        plan.set_params(slrx.make_params(lam=pb.lam, n_irls=args.cpu_outer, n_cg=pb.n_cg, p=pb.p,
                                         gamma=pb.gamma, eps0_frac=pb.eps0_frac))
        plan.run()
        plan.sync()
        out["nrmse_vs_oracle"] = {"value": float(f"{np.linalg.norm(plan.images() - ora) / np.linalg.norm(ora):.3e}"),
                                  "outer_iterations": args.cpu_outer, "bar": 1e-4}
    plan.close()
    if not args.no_extras:
        out["serving"] = measure_serve(120)
        # two warm-up batches: the tuner settles the tridiagonalisation (budget, then
        # row access) and then the CG strategy before the timed batches
        out["batch"] = measure_batch(3, 2, 32, 0.0, check_bits=False)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())

#!/usr/bin/env python3
"""Benchmark: exact Hankel matvecs/s at n = 4096, P = 33220 bits (split-FFT).

Workload (a Lanczos-shaped session): one Hankel matrix with n = 4096 and
h uniform on [-1, 1) at P = 33220 fractional bits is planned once (its 2-D
transform stays resident); then 200 seeded vectors x, each uniform on
[-1, 1) and rescaled to unit 2-norm, are multiplied in turn.  A step is one
planned matvec (limb split + forward limb FFT, index-axis pass against the
resident spectrum, inverse limb FFT + exact carry).  All inputs are resident
in HBM before the timed region starts.

Reported beside the headline: per-step p50/p99 latency, the roofline of the
dominant kernel (from HIP events recorded around each kernel on its stream),
the replay rate of a HIP graph of one step, the exact GPU schoolbook on the
same operands (speedup), and the CPU oracle (Python-int schoolbook) timed on
a bounded row sample on the host cores.

Three further sections report the other workloads of the method (each can be
switched off): the four exact paths on one n = 1024 Hilbert-type product,
the batched launch of 256 uneven products, and the request scheduler under
Poisson arrivals of closed-loop sessions on eight resident matrices.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import random
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Hankel matvecs/s at n=4096, P=33220 bits (split-FFT vs schoolbook); p99 ms"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_cols_pass_n4096_p33220.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1402_5287_amd", "csrc", f)
                  for f in ("fftpath.hip", "fft.h", "fft_layout.h", "common.h")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# (the split-FFT row passes of limb transforms of 3 * 2^k points are
# k_rows_fwd3 / k_rows_inv3, see kernel_names)
KERNEL_NAMES = {"split_fft": ("k_rows_fwd", "k_cols_pass", "k_rows_inv"),
                "ntt": ("k_ntt_rows_fwd", "k_ntt_cols_pass", "k_ntt_rows_inv")}


def kernel_names(algo, info):
    if algo == "split_fft" and info["Nz"] % 3 == 0:
        return ("k_rows_fwd3", "k_cols_pass", "k_rows_inv3")
    return KERNEL_NAMES[algo]


def kernel_bytes(algo, n, W, info):
    """Algorithmic HBM bytes of the three kernels of one planned matvec:
    x words in + X1 spectrum out; X1 in + resident spectrum of h in + Y1 out;
    Y1 in + y words out.  split_fft keeps the Hermitian half (spectrum_cols
    complex binary64 per row: Nz/2 when its two real bins share a column,
    else Nz/2 + 1; the resident spectrum has Nz/2 + 1 columns of Nt), ntt the
    full Nz residues (8 bytes each)."""
    Nt, Nz = info["Nt"], info["Nz"]
    row = info["spectrum_cols"] * 16 if algo == "split_fft" else Nz * 8
    cols = (Nz // 2 + 1) * 16 if algo == "split_fft" else row
    return (n * W * 8 + n * row, 2 * n * row + Nt * cols, n * row + n * W * 8)


def _gen_x(args):
    import seeded_inputs as si
    n, P, k = args
    return si.session_x(n, P, k)


def make_vectors(n, P, count, procs):
    if procs <= 1:
        return [_gen_x((n, P, k)) for k in range(count)]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_gen_x, [(n, P, k) for k in range(count)], chunksize=4)


def host_cpu():
    """nproc, the CPUs this process may use, and lscpu's model line."""
    import subprocess
    out = {"nproc": os.cpu_count(),
           "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "CPU(s)"):
                out[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return out


def _oracle_rows(H, X, P, rows, procs):
    from oracle import hankel
    return hankel.matvec_rows("hankel", H, X, P, rows, processes=procs)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--P", type=int, default=33220)
    ap.add_argument("--vectors", type=int, default=200)
    ap.add_argument("--algo", default="split_fft", choices=("split_fft", "ntt"),
                    help="path of the timed session (the headline is split_fft)")
    ap.add_argument("--no-peer", action="store_true",
                    help="skip timing the NTT path on the same session")
    ap.add_argument("--cpu-rows", type=int, default=24,
                    help="oracle row sample (0 = skip); 24 rows are about 30 s of CPU work")
    ap.add_argument("--no-school", action="store_true", help="skip the GPU schoolbook comparison")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-verify", action="store_true", help="skip the GMP full-vector check")
    ap.add_argument("--no-paths", action="store_true", help="skip the n=1024 four-path section")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-launch section")
    ap.add_argument("--no-serving", action="store_true", help="skip the scheduler section")
    ap.add_argument("--no-lanczos", action="store_true", help="skip the Lanczos section")
    ap.add_argument("--no-float", action="store_true",
                    help="skip the floating-point input section")
    ap.add_argument("--multi", default="2,4,8",
                    help="block sizes k of the multi-vector section (Y = A [x_1..x_k]); "
                         "empty = skip")
    ap.add_argument("--serving-sessions", type=int, default=24)
    ap.add_argument("--serving-loads", default="0.5,0.7,0.9",
                    help="comma-separated offered loads, as fractions of saturated throughput")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--serving-pool-gb", type=float, default=4.5)
    ap.add_argument("--serving-max-large", type=int, default=0,
                    help="large requests in flight at most (0: the server's default policy)")
    ap.add_argument("--serving-large-mb", type=float, default=0.0,
                    help="workspace above which a request is large (with --serving-max-large)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run a plain device copy of BYTES bytes (5 times), the reference "
                         "for scaling hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU layout is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1402_5287_amd import hmv

    n, P, V, K, Wm = args.n, args.P, args.vectors, args.steps, args.warmup
    W = hmv.words(P)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # the host share of one GPU is 16 cores; use them all, never more
    procs = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                       else (os.cpu_count() or 1)))

    if args.copy_calibration > 0:
        a = torch.empty(args.copy_calibration // 8, dtype=torch.int64, device=dev)
        a.fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {args.copy_calibration} bytes")
        del a, b

    t = time.time()
    h = si.session_h(n, P)
    xs_np = make_vectors(n, P, V, procs)
    log(f"inputs generated in {time.time() - t:.1f}s ({V} vectors, {procs} procs)")
    h_dev = hmv.to_device(h, dev)
    xs = torch.from_numpy(np.stack(xs_np).view(np.int64)).to(dev)       # (V, n, W)
    ys = torch.zeros_like(xs)
    torch.cuda.synchronize()

    # ---- plan (once per session)
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_a.record()
    plan = hmv.Plan("hankel", h_dev, n, P, algo=args.algo)
    ev_b.record()
    torch.cuda.synchronize()
    plan_ms = ev_a.elapsed_time(ev_b)
    info = plan.info()
    log(f"plan: w={info['w']} L={info['L']} Nt={info['Nt']} Nz={info['Nz']} "
        f"bound={info['bound']:.3g} variants={info.get('cols_variant')}/"
        f"{info.get('rows_inv_variant')} in {plan_ms:.1f} ms (includes the tuning runs)")

    # ---- warmup
    for k in range(Wm):
        plan.matvec(xs[k % V], ys[k % V])
    torch.cuda.synchronize()

    # ---- timed region: K planned matvecs, events around each kernel
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    for row in evs:
        for e in row:
            e.record()          # creates the underlying HIP events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        plan.matvec_events(xs[k % V], ys[k % V], evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rc, flags, max_err = hmv.read_status(plan.ws)
    if rc != 0 or flags != 0:
        raise SystemExit(f"device status {rc} flags {flags}")

    k1 = [evs[k][0].elapsed_time(evs[k][1]) for k in range(K)]
    k2 = [evs[k][1].elapsed_time(evs[k][2]) for k in range(K)]
    k3 = [evs[k][2].elapsed_time(evs[k][3]) for k in range(K)]
    lat = sorted(evs[k][0].elapsed_time(evs[k][3]) for k in range(K))
    p50 = lat[len(lat) // 2]
    p99 = lat[min(len(lat) - 1, int(0.99 * len(lat)))]
    value = K / wall

    kb = kernel_bytes(args.algo, n, W, info)
    names = kernel_names(args.algo, info)
    kernels = {names[0]: (statistics.mean(k1), kb[0]), names[1]: (statistics.mean(k2), kb[1]),
               names[2]: (statistics.mean(k3), kb[2])}
    bytes_k1, bytes_k2, bytes_k3 = kb
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_ms, dom_bytes = kernels[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = None
    if dom == "k_cols_pass" and args.algo == "split_fft" and os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_sha256") == kernel_source_hash() and tr.get("n") == n and tr.get("P") == P:
            traffic = tr["fetch_bytes"] + tr["write_bytes"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "kernel_ms": round(dom_ms, 4), "algorithmic_bytes": dom_bytes}
    path_bytes = bytes_k1 + bytes_k2 + bytes_k3
    path = {k: {"ms": round(v[0], 4), "GB/s": round(v[1] / (v[0] * 1e-3) / 1e9, 1)}
            for k, v in kernels.items()}
    path["whole_step_roofline_frac"] = round(
        (path_bytes / (HBM_PEAK_GBS * 1e9)) / (wall / K), 4)
    log(f"timed {K} steps in {wall:.3f}s: {value:.1f} matvecs/s, p50 {p50:.3f} ms p99 {p99:.3f} ms")
    log(f"kernels: {path}")

    # ---- graph replay of one step
    graph = None
    if not args.no_graph:
        xg, yg = xs[0].clone(), torch.zeros_like(ys[0])
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(3):
                plan.matvec(xg, yg)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.matvec(xg, yg)
        torch.cuda.synchronize()
        reps = max(K // 2, 50)
        for _ in range(5):
            g.replay()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        gw = time.perf_counter() - tg
        same = bool(torch.equal(yg, ys[0]))
        graph = {"matvecs_per_s": round(reps / gw, 1), "replays": reps, "equal_to_eager": same}
        log(f"graph: {graph}")

    # ---- correctness of the session outputs
    y0 = hmv.to_host(ys[0])
    verify = {}
    if not args.no_verify:
        from oracle import kronecker
        if kronecker.available():
            tv = time.time()
            ok = bool(np.array_equal(y0, kronecker.hankel_matvec_words(h, xs_np[0], P)))
            verify["gmp_full_vector_equal"] = ok
            verify["gmp_seconds"] = round(time.time() - tv, 2)
            log(f"GMP full-vector check: {ok} ({verify['gmp_seconds']} s)")
            if not ok:
                raise SystemExit("split-FFT result differs from the exact product")

    # ---- GPU schoolbook on the same operands: the matrix-core form (the
    # default; one untimed call first) and the binary64 vector form
    school = None
    if not args.no_school:
        ysb = torch.zeros((n, W), dtype=torch.int64, device=dev)
        wsb = hmv.workspace(hmv.oneshot_workspace_bytes("hankel", n, P, "schoolbook"))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def school_ms():
            e0.record()
            hmv.matvec("hankel", h_dev, xs[0], ysb, n, P, algo="schoolbook", ws=wsb)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1)

        school_ms()
        sms = school_ms()
        equal = bool(torch.equal(ysb, ys[0]))
        ysb.zero_()
        hmv.force_school(0)
        try:
            vms = school_ms()
        finally:
            hmv.force_school(-1)
        vequal = bool(torch.equal(ysb, ys[0]))
        school = {"form": "int8 matrix cores", "ms": round(sms, 2),
                  "matvecs_per_s": round(1000.0 / sms, 4),
                  "speedup_split_fft": round(value / (1000.0 / sms), 1),
                  "equal_to_split_fft": equal,
                  "vector_fp64_ms": round(vms, 2),
                  "vector_fp64_equal_to_split_fft": vequal}
        log(f"schoolbook: {school}")
        if not (equal and vequal):
            raise SystemExit("schoolbook and split-FFT disagree")

    # ---- CPU oracle on a bounded row sample
    cpu = None
    if args.cpu_rows > 0:
        from oracle import fixedpoint as fp
        H, X = fp.decode(h), fp.decode(xs_np[0])
        rows = list(range(args.cpu_rows))
        tc = time.perf_counter()
        got = _oracle_rows(H, X, P, rows, procs)
        cw = time.perf_counter() - tc
        same = got == fp.decode(y0[rows])
        cpu = {"value": round((len(rows) / n) / cw, 6), "unit": "matvecs/s", "cores": procs,
               "kind": "oracle",
               "sample": f"{len(rows)} of {n} rows of one matvec (exact Python-int schoolbook, "
                         f"{procs} processes, {cw:.1f} s wall, about {cw * procs:.0f} s of "
                         f"CPU), scaled by rows/n (extrapolated)",
               "host": host_cpu(), "rows_equal_gpu": same}
        log(f"cpu oracle: {cpu}")
        if not same:
            raise SystemExit("oracle rows differ from the GPU result")

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "matvecs/s", "n_gpus": 1,
        "steps": K, "warmup": Wm, "ms_per_step": round(1000.0 * wall / K, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"lanczos-session hankel n={n} P={P}: h uniform[-1,1), "
                               f"{V} unit-norm x, plan once", "n": n, "P": P,
                   "algo": args.algo, "w": info["w"], "L": info["L"], "Nt": info["Nt"],
                   "Nz": info["Nz"], "bound": info["bound"], "vectors": V,
                   "launch_variants": {"index_pass": info.get("cols_variant"),
                                       "inverse_row_pass": info.get("rows_inv_variant")},
                   "parallelism": "single-gpu"},
        "p50_ms": round(p50, 4), "p99_ms": round(p99, 4), "plan_ms": round(plan_ms, 2),
        "max_round_err": max_err,
        "roofline": roofline, "kernels": path, "graph": graph, "schoolbook_gpu": school,
        "verify": verify, "cpu_baseline": cpu,
        "ntt_peer": None if (args.no_peer or args.algo != "split_fft")
        else section_peer(dev, plan, h_dev, xs, ys, n, P, W, K, Wm),
        "multi_vector": None if (not args.multi or args.algo != "split_fft")
        else section_multi(plan, xs, ys, n, W, info, [int(k) for k in args.multi.split(",")],
                           K),
        "lanczos": None if args.no_lanczos else section_lanczos(dev),
        "float_inputs": None if args.no_float else section_float(dev, h_dev, xs, n, P),
        "paths_n1024": None if args.no_paths else section_paths(dev),
        "batch": None if args.no_batch else section_batch(dev),
        "serving": None if args.no_serving else section_serving(dev, procs, args),
    }
    print(json.dumps(out), flush=True)


def section_peer(dev, fplan, h_dev, xs, ys, n, P, W, K, Wm):
    """The exact NTT path on the same session: rate, kernels, and equality
    with the split-FFT outputs."""
    import torch

    from paper_1402_5287_amd import hmv
    V = xs.shape[0]
    plan = hmv.Plan("hankel", h_dev, n, P, algo="ntt")
    info = plan.info()
    yn = torch.zeros_like(ys[0])
    for k in range(Wm):
        plan.matvec(xs[k % V], yn)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    for row in evs:
        for e in row:
            e.record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        plan.matvec_events(xs[k % V], yn, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    same = bool(torch.equal(yn, ys[(K - 1) % V]))
    plan.matvec(xs[0], yn)
    torch.cuda.synchronize()
    same = same and bool(torch.equal(yn, ys[0]))
    kb = kernel_bytes("ntt", n, W, info)
    ks = {}
    for j, name in enumerate(KERNEL_NAMES["ntt"]):
        ms = statistics.mean(evs[k][j].elapsed_time(evs[k][j + 1]) for k in range(K))
        ks[name] = {"ms": round(ms, 4), "GB/s": round(kb[j] / (ms * 1e-3) / 1e9, 1)}
    lat = sorted(evs[k][0].elapsed_time(evs[k][3]) for k in range(K))
    res = {"matvecs_per_s": round(K / wall, 1), "p50_ms": round(lat[len(lat) // 2], 4),
           "p99_ms": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4),
           "w": info["w"], "L": info["L"], "Nt": info["Nt"], "Nz": info["Nz"],
           "plan_mb": round(info["plan_bytes"] / 2**20, 1), "kernels": ks,
           "equal_to_split_fft": same}
    log(f"ntt peer: {res}")
    plan.close()
    if not same:
        raise SystemExit("NTT and split-FFT sessions disagree")
    return res


def section_multi(plan, xs, ys, n, W, info, ks, K):
    """Blocks of k session vectors with the one plan (Y = A [x_1 .. x_k]):
    matvecs/s, per-pass times per block, the index-axis pass's algorithmic
    bytes per matvec (spectra of x and y per vector, the resident spectrum
    once per block), and equality with the single-vector outputs."""
    import torch

    V = xs.shape[0]
    Vf = min(V, K)               # vectors whose single-vector outputs ys holds
    res = {}
    kb = kernel_bytes("split_fft", n, W, info)
    row = info["spectrum_cols"] * 16
    h_bytes = kb[1] - 2 * n * row
    for k in ks:
        if k < 1 or k > Vf:
            continue
        ws = plan.multi_workspace(k)
        nb = max(4, K // (2 * k))
        blocks = [(j * k) % (Vf - k + 1) for j in range(nb)]
        flat_x = xs.reshape(V * n, W)
        yb = torch.zeros((k * n, W), dtype=torch.int64, device=xs.device)
        for j in range(2):
            b0 = blocks[j]
            plan.matvec_multi(flat_x[b0 * n:(b0 + k) * n], yb, k, ws)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nb)]
        for r in evs:
            for e in r:
                e.record()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j, b0 in enumerate(blocks):
            plan.matvec_multi(flat_x[b0 * n:(b0 + k) * n], yb, k, ws, events=evs[j])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        b0 = blocks[-1]
        same = bool(torch.equal(yb.reshape(k, n, W), ys[b0:b0 + k]))
        per = [statistics.mean(evs[j][q].elapsed_time(evs[j][q + 1]) for j in range(nb))
               for q in range(3)]
        cols_bytes = 2 * n * row + h_bytes / k          # per matvec
        res[str(k)] = {
            "matvecs_per_s": round(nb * k / wall, 1),
            "ms_per_block": round(1000.0 * wall / nb, 4),
            "kernels_ms_per_matvec": {nm: round(t / k, 4) for nm, t in
                                      zip(kernel_names("split_fft", info), per)},
            "cols_pass_alg_bytes_per_matvec": int(cols_bytes),
            "cols_pass_GB_s": round(cols_bytes * k / (per[1] * 1e-3) / 1e9, 1),
            "equal_to_single": same}
        log(f"multi k={k}: {res[str(k)]}")
        if not same:
            raise SystemExit("block product differs from the single-vector products")
        del ws
    return res


def section_lanczos(dev, steps=20):
    """The Lanczos tridiagonalisation (hmv_lanczos) over planned matvecs at
    the paper's Lanczos sizes (n = 100) and at n = 1024, P = 33220: time per
    step, and the share of the matvec in it."""
    import torch

    import seeded_inputs as si
    from paper_1402_5287_amd import hmv
    res = {}
    for n in (100, 1024):
        P = 33220
        h = si.uniform(2 * n - 1, P, (6, 0, n))
        q1 = hmv.to_device(si.unit_norm(si.uniform(n, P, (6, 1, n)), P), dev)
        plan = hmv.Plan("hankel", hmv.to_device(h, dev), n, P, algo="split_fft")
        plan.lanczos(q1, 2)                                 # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        alpha, beta, done, _, ws = plan.lanczos(q1, steps)
        e1.record()
        torch.cuda.synchronize()
        rc, flags, _ = hmv.read_status(ws)
        ms = e0.elapsed_time(e1)
        y = torch.zeros_like(q1)
        m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        m0.record()
        for _ in range(steps):
            plan.matvec(q1, y)
        m1.record()
        torch.cuda.synchronize()
        mv = m0.elapsed_time(m1) / steps
        done_k = int(done.item())
        res[str(n)] = {"P": P, "steps": done_k, "ms_per_step": round(ms / max(1, done_k), 3),
                       "matvec_ms": round(mv, 4), "status": rc, "flags": flags}
        log(f"lanczos n={n}: {res[str(n)]}")
        plan.close()
    return res


def section_float(dev, h_words, xs, n, P, spread=64, steps=50):
    """Floating-point inputs (hmv_fplan_*) at the headline shape: the session's
    words as P-bit significands with seeded exponents spread over `spread`
    bits; matvecs/s of the floating plan (fixed point at Q = P + spread bits
    inside) next to the plain fixed-point plan at Q bits."""
    import numpy as np
    import torch

    from paper_1402_5287_amd import hmv
    rng = np.random.default_rng(7)
    hl = h_words.shape[0]
    he = torch.from_numpy(rng.integers(-spread, 1, size=hl).astype(np.int32)).to(dev)
    xe = torch.from_numpy(rng.integers(-spread, 1, size=(xs.shape[0], n)).astype(np.int32)).to(dev)
    t0 = time.time()
    fplan = hmv.FPlan("hankel", h_words, he, n, P, spread)
    torch.cuda.synchronize()
    plan_ms = (time.time() - t0) * 1000
    W = hmv.words(P)
    ys = torch.zeros((n, W), dtype=torch.int64, device=dev)
    ye = torch.zeros(n, dtype=torch.int32, device=dev)
    for k in range(3):
        fplan.matvec(xs[k % xs.shape[0]], xe[k % xs.shape[0]], ys, ye)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        fplan.matvec(xs[k % xs.shape[0]], xe[k % xs.shape[0]], ys, ye)
    e1.record()
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1) / steps
    rc, flags, _ = hmv.read_status(fplan.ws)
    info = fplan.info()
    fplan.close()
    # the fixed-point plan at the same inner precision Q
    Q = info["Q"]
    WQ = hmv.words(Q)
    hq = torch.zeros((hl, WQ), dtype=torch.int64, device=dev)
    hq[:, :W] = h_words
    hq[:, W:] = torch.where(h_words[:, W - 1:W] < 0, -1, 0)
    xq = torch.zeros((n, WQ), dtype=torch.int64, device=dev)
    xq[:, :W] = xs[0]
    xq[:, W:] = torch.where(xs[0][:, W - 1:W] < 0, -1, 0)
    qplan = hmv.Plan("hankel", hq, n, Q, algo="split_fft")
    yq = torch.zeros_like(xq)
    for _ in range(3):
        qplan.matvec(xq, yq)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        qplan.matvec(xq, yq)
    e1.record()
    torch.cuda.synchronize()
    qms = e0.elapsed_time(e1) / steps
    qplan.close()
    res = {"n": n, "P": P, "spread": spread, "Q": Q, "plan_ms": round(plan_ms, 1),
           "matvec_ms": round(fms, 4), "matvecs_per_s": round(1000.0 / fms, 1),
           "fixed_point_Q_matvec_ms": round(qms, 4), "status": rc, "flags": flags,
           "w": info["w"], "Nz": info["Nz"]}
    log(f"float inputs: {res}")
    if rc != 0 or flags:
        raise SystemExit("floating-point matvec reported a nonzero status")
    return res


def _ms_between(e0, e1):
    return e0.elapsed_time(e1)


def section_paths(dev, reps=5):
    """Four exact paths on the n = 1024, P = 33220 Hilbert-type product; every
    result must equal every other and the exact CPU product."""
    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1402_5287_amd import hmv
    n, P = 1024, 33220
    h, x = si.hilbert_case(n, P)
    hd, xd = hmv.to_device(h, dev), hmv.to_device(x, dev)
    res, outs = {}, {}
    for algo in ("split_fft", "ntt", "karatsuba"):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        plan = hmv.Plan("hankel", hd, n, P, algo=algo)
        e[1].record()
        y = torch.zeros_like(xd)
        plan.matvec(xd, y)
        torch.cuda.synchronize()
        e[2].record()
        for _ in range(reps):
            plan.matvec(xd, y)
        e[3].record()
        torch.cuda.synchronize()
        info = plan.info()
        res[algo] = {"plan_ms": round(_ms_between(e[0], e[1]), 3),
                     "matvec_ms": round(_ms_between(e[2], e[3]) / reps, 4),
                     "w": info["w"], "L": info["L"], "Nt": info["Nt"], "Nz": info["Nz"]}
        outs[algo] = y
        plan.close()
        log(f"paths n=1024 {algo}: {res[algo]}")
    ys = torch.zeros_like(xd)
    ws = hmv.workspace(hmv.oneshot_workspace_bytes("hankel", n, P, "schoolbook"), device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    hmv.matvec("hankel", hd, xd, ys, n, P, algo="schoolbook", ws=ws)
    e1.record()
    torch.cuda.synchronize()
    res["schoolbook"] = {"matvec_ms": round(_ms_between(e0, e1), 3)}
    log(f"paths n=1024 schoolbook: {res['schoolbook']}")
    outs["schoolbook"] = ys
    equal = all(torch.equal(outs[a], ys) for a in outs)
    res["all_equal"] = bool(equal)
    from oracle import kronecker
    if kronecker.available():
        res["equal_exact_cpu"] = bool(np.array_equal(hmv.to_host(ys),
                                                     kronecker.hankel_matvec_words(h, x, P)))
    if not equal or not res.get("equal_exact_cpu", True):
        raise SystemExit(f"n=1024 paths disagree: {res}")
    sb = res["schoolbook"]["matvec_ms"]
    for a in ("split_fft", "ntt", "karatsuba"):
        res[a]["speedup_vs_schoolbook"] = round(sb / res[a]["matvec_ms"], 1)
    return res


def section_batch(dev, count=256, reps=3):
    """256 uneven (kind, n, P) products in the batched launch, checked against
    the single-product path one by one."""
    import torch

    import seeded_inputs as si
    from paper_1402_5287_amd import hmv
    t = time.time()
    inst = si.batch_instances(count)
    items, hs, xs = [], [], []
    for i, (kind, n, P) in enumerate(inst):
        h, x = si.batch_operands(i, kind, n, P)
        hd, xd = hmv.to_device(h, dev), hmv.to_device(x, dev)
        yd = torch.zeros_like(xd)
        items.append((kind, hd, xd, yd, n, P))
    log(f"batch: {count} instances generated in {time.time() - t:.1f}s")
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_workspace_bytes(probs), device=dev)
    hmv.batch_matvec(probs, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        hmv.batch_matvec(probs, ws)
    e1.record()
    torch.cuda.synchronize()
    bms = _ms_between(e0, e1) / reps
    # the same batch in one cooperative launch: timed, outputs compared
    ref = [it[3].clone() for it in items]
    batch_mb = ws.numel() / 2**20
    _, batch_flags, _ = hmv.read_status(ws)
    del ws
    ws = hmv.workspace(hmv.batch_single_workspace_bytes(probs), device=dev)
    single_mb = ws.numel() / 2**20
    hmv.batch_matvec_single(probs, ws)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        hmv.batch_matvec_single(probs, ws)
    e1.record()
    torch.cuda.synchronize()
    one_ms = _ms_between(e0, e1) / reps
    one_equal = all(torch.equal(r, it[3]) for r, it in zip(ref, items))
    # the same products one at a time (one-shot auto path), timed and compared
    single_ws = hmv.workspace(max(hmv.oneshot_workspace_bytes(k, n, P) for (k, _, _, _, n, P)
                                  in items), device=dev)
    outs = []
    e0.record()
    for (kind, hd, xd, yd, n, P) in items:
        y1 = torch.zeros_like(yd)
        hmv.matvec(kind, hd, xd, y1, n, P, ws=single_ws)
        outs.append(y1)
    e1.record()
    torch.cuda.synchronize()
    sms = _ms_between(e0, e1)
    equal = all(torch.equal(o, it[3]) for o, it in zip(outs, items))
    rc, flags, _ = hmv.read_status(ws)
    flags |= batch_flags
    res = {"instances": count, "launches": hmv.batch_launches(probs), "batch_ms": round(bms, 3),
           "products_per_s": round(count / (bms * 1e-3), 1),
           "one_launch_ms": round(one_ms, 3),
           "one_launch_products_per_s": round(count / (one_ms * 1e-3), 1),
           "one_launch_equal": bool(one_equal),
           "one_launch_workspace_mb": round(single_mb, 1),
           "one_by_one_ms": round(sms, 3), "equal_to_single_path": bool(equal),
           "status_flags": flags,
           "kinds": [sum(1 for k, _, _ in inst if k == c) for c in range(3)],
           "workspace_mb": round(batch_mb, 1)}
    log(f"batch: {res}")
    if not equal or not one_equal or flags:
        raise SystemExit("batched products differ from the single path")
    return res


def _serve_vectors(args):
    import seeded_inputs as si
    m, n, P, j = args
    return si.serving_x(m, n, P, j)


def section_serving(dev, procs, args, pool_vectors=4):
    """Poisson arrivals of closed-loop sessions on 8 resident matrices through
    the request scheduler: matvecs/s and request latency p50/p99."""
    import multiprocessing as mp

    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1402_5287_amd import hmv, serving
    t = time.time()
    mats = si.serving_matrices()
    plans = []
    for m, (n, P) in enumerate(mats):
        plans.append(hmv.Plan("hankel", hmv.to_device(si.serving_h(m, n, P), dev), n, P))
    jobs = [(m, n, P, j) for m, (n, P) in enumerate(mats) for j in range(pool_vectors)]
    with mp.get_context("fork").Pool(procs) as pool:
        vecs = pool.map(_serve_vectors, jobs)
    xpool = {}
    for (m, n, P, j), v in zip(jobs, vecs):
        xpool[(m, j)] = hmv.to_device(v, dev)
    torch.cuda.synchronize()
    log(f"serving: {len(mats)} plans + {len(jobs)} vectors ready in {time.time() - t:.1f}s")
    W = hmv.words(mats[0][1])
    ws_need = [p.mv_ws_bytes for p in plans]
    pool_bytes = int(args.serving_pool_gb * 2**30)
    info = [p.info() for p in plans]

    def make_sessions(desc, arrivals, base):
        out = []
        for sid, ((m, length), arr) in enumerate(zip(desc, arrivals)):
            n = mats[m][0]
            y = torch.zeros((n, W), dtype=torch.int64, device=dev)
            xs = [xpool[(m, (sid + k) % pool_vectors)] for k in range(length)]
            out.append(serving.Session(sid=base + sid, matrix_id=m, arrival=arr, xs=xs,
                                       ys=[y] * length))
        return out

    def drive(sessions):
        server = hmv.Server(pool_bytes, slots=args.serving_slots, device=dev)
        for p in plans:
            server.add_plan(p)
        if args.serving_max_large > 0:
            server.set_policy(int(args.serving_large_mb * 2**20), args.serving_max_large)
        wall, lats, recs = serving.run(server, sessions, time_limit=300.0)
        torch.cuda.synchronize()
        st = server.stats()
        server.close()
        if any(r[3] != 0 for r in recs):
            raise SystemExit("serving: a request reported a nonzero status")
        return wall, lats, st

    # saturated throughput: every session present at t = 0
    sat_desc = [(m % len(mats), 30) for m in range(2 * len(mats))]
    sat = make_sessions(sat_desc, [0.0] * len(sat_desc), 0)
    wall, lats, st = drive(sat)
    sat_rate = sum(len(s.xs) for s in sat) / wall
    log(f"serving: saturated {sat_rate:.1f} matvecs/s ({wall:.2f}s, max in flight "
        f"{st['max_in_flight']})")
    res = {"matrices": [{"n": n, "P": P, "w": i["w"], "Nt": i["Nt"], "Nz": i["Nz"],
                         "workspace_mb": round(b / 2**20, 1)}
                        for (n, P), i, b in zip(mats, info, ws_need)],
           "slots": args.serving_slots, "pool_gb": args.serving_pool_gb,
           "policy": {"large_mb": round(st["large_bytes"] / 2**20, 1),
                      "max_large": st["max_large"]},
           "saturated_matvecs_per_s": round(sat_rate, 1), "loads": []}
    for li, load in enumerate(float(v) for v in args.serving_loads.split(",")):
        desc = si.serving_sessions(args.serving_sessions, len(mats), seed=li)
        mean_len = sum(d[1] for d in desc) / len(desc)
        lam = load * sat_rate / mean_len
        arrivals = serving.poisson_arrivals(lam, len(desc), random.Random(1000 + li))
        sess = make_sessions(desc, arrivals, 10000 * (li + 1))
        wall, lats, st = drive(sess)
        total = sum(len(s.xs) for s in sess)
        by_n = {}
        for s in sess:
            by_n.setdefault(mats[s.matrix_id][0], []).extend(s.latencies)
        # every session's last result against the same product run alone
        same = True
        for s in sess:
            p = plans[s.matrix_id]
            alone = torch.zeros_like(s.ys[-1])
            p.matvec(s.xs[-1], alone, ws=p.new_workspace())
            torch.cuda.synchronize()
            same = same and bool(torch.equal(alone, s.ys[-1]))
        ent = {"load": load, "sessions": len(sess), "arrival_rate_per_s": round(lam, 3),
               "matvecs": total, "wall_s": round(wall, 3),
               "matvecs_per_s": round(total / wall, 1),
               "p50_ms": round(1e3 * serving.percentile(lats, 0.5), 3),
               "p99_ms": round(1e3 * serving.percentile(lats, 0.99), 3),
               "by_n": {str(n): {"p50_ms": round(1e3 * serving.percentile(v, 0.5), 3),
                                 "p99_ms": round(1e3 * serving.percentile(v, 0.99), 3),
                                 "count": len(v)} for n, v in sorted(by_n.items())},
               "max_in_flight": st["max_in_flight"],
               "max_large_in_flight": st["max_large_in_flight"],
               "pool_peak_mb": round(st["pool_peak"] / 2**20, 1),
               "last_results_equal_alone": same}
        log(f"serving load {load}: {ent}")
        if not same:
            raise SystemExit("serving: a result in the mix differs from the same product alone")
        res["loads"].append(ent)
    for p in plans:
        p.close()
    return res


if __name__ == "__main__":
    main()

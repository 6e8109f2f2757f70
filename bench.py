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
    ap.add_argument("--cpu-rows", type=int, default=16, help="oracle row sample (0 = skip)")
    ap.add_argument("--no-school", action="store_true", help="skip the GPU schoolbook comparison")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-verify", action="store_true", help="skip the GMP full-vector check")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run a plain device copy of BYTES bytes (5 times), the reference "
                         "for scaling hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU layout is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import seeded_inputs as si
    from paper_1402_5287_amd import hmv

    n, P, V, K, Wm = args.n, args.P, args.vectors, args.steps, args.warmup
    W = hmv.words(P)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    procs = max(1, min(16, os.cpu_count() or 1))

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
    plan = hmv.Plan("hankel", h_dev, n, P, algo="split_fft")
    ev_b.record()
    torch.cuda.synchronize()
    plan_ms = ev_a.elapsed_time(ev_b)
    info = plan.info()
    log(f"plan: w={info['w']} L={info['L']} Nt={info['Nt']} Nz={info['Nz']} "
        f"bound={info['bound']:.3g} in {plan_ms:.1f} ms")

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

    C = info["Nz"] // 2 + 1
    Nt = info["Nt"]
    bytes_k1 = n * W * 8 + n * C * 16
    bytes_k2 = 2 * n * C * 16 + C * Nt * 16
    bytes_k3 = n * C * 16 + n * W * 8
    kernels = {
        "k_rows_fwd": (statistics.mean(k1), bytes_k1),
        "k_cols_pass": (statistics.mean(k2), bytes_k2),
        "k_rows_inv": (statistics.mean(k3), bytes_k3),
    }
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_ms, dom_bytes = kernels[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = None
    if dom == "k_cols_pass" and os.path.exists(TRAFFIC_FILE):
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

    # ---- GPU schoolbook on the same operands
    school = None
    if not args.no_school:
        ysb = torch.zeros((n, W), dtype=torch.int64, device=dev)
        wsb = hmv.workspace(hmv.oneshot_workspace_bytes("hankel", n, P, "schoolbook"))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        hmv.matvec("hankel", h_dev, xs[0], ysb, n, P, algo="schoolbook", ws=wsb)
        e1.record()
        torch.cuda.synchronize()
        sms = e0.elapsed_time(e1)
        school = {"ms": round(sms, 2), "matvecs_per_s": round(1000.0 / sms, 4),
                  "speedup_split_fft": round((1000.0 / sms and value / (1000.0 / sms)), 1),
                  "equal_to_split_fft": bool(torch.equal(ysb, ys[0]))}
        log(f"schoolbook: {school}")
        if not school["equal_to_split_fft"]:
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
                         f"{procs} processes, {cw:.1f} s wall), scaled by rows/n",
               "rows_equal_gpu": same}
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
                   "algo": "split_fft", "w": info["w"], "L": info["L"], "Nt": info["Nt"],
                   "Nz": info["Nz"], "bound": info["bound"], "vectors": V,
                   "parallelism": "single-gpu"},
        "p50_ms": round(p50, 4), "p99_ms": round(p99, 4), "plan_ms": round(plan_ms, 2),
        "max_round_err": max_err,
        "roofline": roofline, "kernels": path, "graph": graph, "schoolbook_gpu": school,
        "verify": verify, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

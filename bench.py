#!/usr/bin/env python3
"""Benchmark of the randomized SVD (Algorithm 4) on one MI355X.

A step is one complete solve (Omega generation, sketch, q re-orthonormalised
power iterations, projection, small SVD, lift, signs) of the workload's
matrix, which is resident in HBM before the timed region starts.  The
default workload is the FP32 configuration: A = U diag(max(0.95^i, 1e-6)) V^T,
8192 x 8192, Haar U and V, k = 100, p = 10, q = 2, Philox seed 0.

Prints one JSON line: solves/s, ms per solve, p50/p99 latency, algorithmic
TFLOP/s, the accuracy against the FP64 oracle, the roofline of the dominant
kernel (timed with HIP events on the solve's stream) and the FP64 CPU
oracle's own rate on this host.  After the default workload the same line
carries the single-pass Algorithm 6 on the same matrix (its two-sided sketch
kernel's roofline) and the mixed-precision workload's three storage forms.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RSVD solves/s + MFMA TFLOP/s at fixed rel. error vs FP64; p50/p99 latency"
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}      # MI355X dense MFMA peaks
PEAK_VALU_TFLOPS = {"f32": 157.3, "f64": 78.6}  # MI355X vector peaks
HBM_PEAK_GBS = 8000.0                          # MI355X HBM3E
LP_KIND_NAMES = {0: "sketch A*Omega (lp_gemm_kernel<AB,false,true,LT>)",
                 1: "A*W (lp_gemm_kernel<AB,false,false,LT>)",
                 2: "A^T*Q (lp_gemm_kernel<AB,true,false,LT>)"}
KIND_NAMES = {0: "sketch A*Omega (skinny_gemm_kernel<float,false,true,LT>)",
              1: "A*W (skinny_gemm_kernel<float,false,false,LT>)",
              2: "A^T*Q (skinny_gemm_kernel<float,true,false,LT>)"}


def _describe(name, cfg):
    kind = cfg["spectrum"]
    if kind[0] == "geometric":
        spec = f"sigma_i=max({kind[1]}^i,{kind[2]:g})" if kind[2] else f"sigma_i={kind[1]}^i"
    elif kind[0] == "power":
        spec = f"sigma_i=i^-{kind[1]:g}"
    else:
        spec = "60 Gaussian bumps + N(0,0.05^2) noise"
    return (f"{name}: A {cfg['m']}x{cfg['n']} {cfg['dtype']}, {spec}, Haar U,V (numpy PCG64 seeds 1,2); "
            f"k={cfg['k']} p={cfg['p']} q={cfg['q']}; Philox Omega seed 0")


def _cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) for the oracle baseline."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([d.get("num_threads", 1) for d in threadpool_info()] or [1]))
    except Exception:
        return len(os.sched_getaffinity(0))


def _oracle_single_thread(Ah, k, p, q, budget_s=10.0):
    """Whole FP64 oracle solves with one BLAS thread, for the small
    configurations: solves/s and the number of solves timed."""
    from threadpoolctl import threadpool_limits
    from oracle.rsvd import rsvd_alg4
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        n = 0
        while True:
            rsvd_alg4(Ah, k, p, q, seed=0)
            n += 1
            if time.perf_counter() - t0 >= budget_s or n >= 200:
                break
        return n / (time.perf_counter() - t0), n


def _jacobi_flops(l, sweeps):
    """Algorithmic work of the small SVD's one-sided Jacobi iteration on the
    l x l factor: per pair and sweep one inner product (2 l flops) and the
    update of the two columns (4 l flops), l (l - 1) / 2 pairs per sweep."""
    return float(sweeps) * l * (l - 1) / 2.0 * 6.0 * l


def _time_solver(torch, solver, steps, warmup):
    for _ in range(warmup):
        solver()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record()
        solver()
        evs[i][1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, np.array([a.elapsed_time(b) for a, b in evs])


def bench_lowp(args, cfg, A, torch, rsvd, workloads):
    """The mixed-precision workload: the same FP32 matrix solved in FP32, and
    stored in BF16 and in column-scaled FP8 (power iterations on the stored
    A with one extra pass, Rayleigh-Ritz projection on the FP32 copy).  The
    headline value is the BF16 form; every form carries its own roofline and
    its error against the FP64 oracle on the FP32 matrix."""
    m, n, k, p, q = cfg["m"], cfg["n"], cfg["k"], cfg["p"], cfg["q"]
    dev = A.device
    forms = {}
    stored = {}                                   # the low-precision copies, for the oracle leg
    for name in ("f32", "bf16", "fp8"):
        M = A if name == "f32" else rsvd.quantize(A, rsvd.RSVD_BF16 if name == "bf16" else rsvd.RSVD_FP8_E4M3)
        if name != "f32" and not args.no_cpu_baseline:
            stored[name] = (M.data.cpu().numpy(), M.col_scale.cpu().numpy() if M.col_scale is not None else None)
        solver = rsvd.Solver(M, k, p, q, seed=0)
        l = solver.l
        dt, lat = _time_solver(torch, solver, args.steps, args.warmup)
        rsvd.profile_enable(dev, True)
        for _ in range(max(2, args.steps // 4)):
            solver()
        torch.cuda.synchronize()
        rsvd.profile_enable(dev, False)
        kinds = {}
        for kind in (0, 1, 2, 4):
            tot, cnt = rsvd.profile_read(dev, kind)
            if cnt:
                kinds[kind] = (tot, cnt)
        st1_tot, st1_cnt = rsvd.profile_read(dev, rsvd.PROFILE_STAGE1)
        lp_kinds = [kk for kk in kinds if kk != 4]
        dom = max(lp_kinds, key=lambda kk: kinds[kk][0])
        dom_ms = kinds[dom][0] / kinds[dom][1]
        if name == "f32":
            achieved = 2.0 * m * n * l / (dom_ms * 1e-3) / 1e12
            roof = {"bound": "mfma", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s", "frac": achieved / 157.3}
        else:
            nbytes = m * n * (2 if name == "bf16" else 1)
            achieved = nbytes / (dom_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": float(nbytes)}
        kname = KIND_NAMES[dom] if name == "f32" else LP_KIND_NAMES[dom].replace("AB", "2" if name == "bf16" else "1")
        roof.update({"kernel": kname,
                     "avg_launch_ms": dom_ms, "launches_per_solve": kinds[dom][1] / max(2, args.steps // 4),
                     "traffic": None})
        if 4 in kinds:
            roof["fp32_projection_ms"] = kinds[4][0] / kinds[4][1]
        forms[name] = {"solves_per_s": args.steps / dt, "ms_per_step": dt / args.steps * 1e3,
                       "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                       "power_iterations": q + (0 if name == "f32" else 1), "info": int(solver.info.item()),
                       "range_finder_ms": st1_tot / max(1, st1_cnt),
                       "S": solver.S.cpu().numpy(), "roofline": roof}
        print(f"bench: {name}: {forms[name]['ms_per_step']:.2f} ms per solve", file=sys.stderr, flush=True)
        del solver, M
        torch.cuda.empty_cache()
    sig = workloads.config_sigma(args.config)
    for f in forms.values():
        f["err_vs_true_spectrum_normwise"] = float(np.max(np.abs(f["S"] - sig[:k])) / sig[0])
    out = {
        "metric": METRIC, "value": forms["bf16"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": forms["bf16"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": _describe(args.config, cfg) + "; stored in BF16 (headline), FP8 E4M3 with column "
                   "scales, and FP32; one extra power iteration for BF16/FP8; FP32 Rayleigh-Ritz",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "l": rsvd.l_used(m, n, k, p)},
        "p50_ms": forms["bf16"]["p50_ms"], "p99_ms": forms["bf16"]["p99_ms"],
        "roofline": forms["bf16"]["roofline"],
    }
    if not args.no_cpu_baseline:
        # Errors against the FP64 oracle, per form: on the FP32 master (cast to
        # FP64) with the form's own number of power iterations, and for BF16
        # and FP8 also on the dequantized stored matrix.
        from oracle.quant import dequantize_bf16, dequantize_fp8
        from oracle.rsvd import rsvd_alg4

        def errs(S, ref):
            return {"sigma_normwise_max": float(np.max(np.abs(S - ref["S"])) / ref["S"][0]),
                    "sigma_relative_max": float(np.max(np.abs(S - ref["S"]) / ref["S"]))}

        Ah = A.double().cpu().numpy()
        print("bench: FP64 CPU oracle on the FP32 matrix ...", file=sys.stderr, flush=True)
        tc = time.perf_counter()
        ref = rsvd_alg4(Ah, k, p, q, seed=0)
        tcpu = time.perf_counter() - tc
        out["cpu_baseline"] = {"value": 1.0 / tcpu, "unit": "solves/s", "cores": _blas_threads(), "kind": "oracle",
                               "sample": f"1 full FP64 solve of the same workload ({m}x{n}, k={k}, p={p}, q={q}), "
                                         f"{tcpu:.1f} s wall clock incl. Omega generation",
                               "cpu_model": _cpu_model()}
        forms["f32"]["rel_err_vs_fp64_oracle"] = errs(forms["f32"]["S"], ref)
        print(f"bench: oracle {tcpu:.1f} s; with q = {q + 1} ...", file=sys.stderr, flush=True)
        ref1 = rsvd_alg4(Ah, k, p, q + 1, seed=0)
        del Ah
        for name in ("bf16", "fp8"):
            data, scale = stored.pop(name)
            print(f"bench: FP64 CPU oracle on the dequantized {name} matrix ...", file=sys.stderr, flush=True)
            Ad = dequantize_bf16(data.view(np.uint16)) if name == "bf16" else dequantize_fp8(data, scale)
            del data
            refd = rsvd_alg4(Ad, k, p, q + 1, seed=0)
            del Ad
            forms[name]["rel_err_vs_fp64_oracle_master"] = errs(forms[name]["S"], ref1)
            forms[name]["rel_err_vs_fp64_oracle_dequantized"] = errs(forms[name]["S"], refd)
    for f in forms.values():
        del f["S"]
    out["forms"] = forms
    return out


def bench_single_pass(args, A, cfg, torch, rsvd, prof_summary, with_oracle):
    """Algorithm 6 (single pass) on the same matrix: solves/s, and the
    two-sided sketch kernel (A Omega_c and A^T Omega_r from one read of A)
    against the FP32/FP64 MFMA peak, with the oracle's sigma error."""
    m, n, k, p = cfg["m"], cfg["n"], cfg["k"], cfg["p"]
    dev = A.device
    solver = rsvd.Solver(A, k, p, 0, seed=0, algorithm=6)
    l = solver.l
    for _ in range(args.warmup):
        solver()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    rsvd.profile_enable(dev, True)
    for _ in range(args.steps):
        solver()
    torch.cuda.synchronize()
    rsvd.profile_enable(dev, False)
    d_tot, d_cnt = rsvd.profile_read(dev, rsvd.PROFILE_DUAL)
    s_tot, s_cnt = rsvd.profile_read(dev, rsvd.PROFILE_STAGE1)
    j_tot, j_cnt = rsvd.profile_read(dev, rsvd.PROFILE_JACOBI)
    rsvd.profile_read(dev, rsvd.PROFILE_ALL)
    d_ms = d_tot / max(1, d_cnt)
    flops = 2 * 2.0 * m * n * l
    ach = flops / (d_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[cfg["dtype"]]
    out = {
        "algorithm": 6, "solves_per_s": 1.0 / dt, "ms_per_solve": dt * 1e3, "l": l,
        "info": int(solver.info.item()),
        "two_sided_sketch": {"kernel": "dual_sketch_kernel<float,%d>" % ((l + 15) // 16), "avg_launch_ms": d_ms,
                             "flops_per_launch": flops, "achieved_tflops": ach, "peak_tflops": peak,
                             "frac": ach / peak, "a_bytes_read_once": float(m * n * A.element_size()),
                             "note": "A Omega_c and A^T Omega_r (2 x 2mnl flops) from one read of A; its row-tile "
                                     "partials of A^T Omega_r are reduced by a separate kernel (outside this time)"},
        "stage1_ms": s_tot / max(1, s_cnt),
        "small_svds_ms": j_tot / max(1, args.steps),
        "small_svds_per_solve": j_cnt / max(1, args.steps),
    }
    # HBM bytes per launch from the committed counter summary, while the
    # kernel's source is the one the counters measured.
    tr = prof_summary.read_traffic(os.path.join(ROOT, "profiles", "dual_sketch_c2_fp32_8192_traffic.txt"))
    out["two_sided_sketch"]["traffic"] = tr[0] if tr is not None and tr[1] == prof_summary.gemm_source_hash("dual") \
        else None
    if with_oracle:
        from oracle.single_pass import rsvd_alg6
        ref = rsvd_alg6(A.double().cpu().numpy(), k, p, seed=0)
        S = solver.S.cpu().numpy()
        out["rel_err_vs_fp64_oracle_sigma_normwise"] = float(np.max(np.abs(S - ref["S"])) / ref["S"][0])
    del solver
    return out


def bench_serving(args, cfg, torch, rsvd, workloads):
    """The serving workload through the request server: a Poisson replay of
    the trace (latency percentiles at the offered load), then a saturation
    replay (every request submitted at once: peak solves/s, the headline),
    the alone-vs-mix identity of every result, and the FP64 oracle on a
    sample of requests."""
    dev = torch.device("cuda:0")
    torch.backends.cuda.matmul.allow_tf32 = False
    trace = workloads.serving_trace(cfg["count"], cfg["rate"])
    print(f"bench: building {len(trace)} request matrices ...", file=sys.stderr, flush=True)
    tg = time.perf_counter()
    pool = workloads.HaarPool(dev, sorted({r["m"] for r in trace} | {r["n"] for r in trace}))
    mats = [pool.matrix(r) for r in trace]
    del pool
    torch.cuda.synchronize()
    print(f"bench: inputs ready in {time.perf_counter() - tg:.1f} s", file=sys.stderr, flush=True)
    budget = int(cfg["budget_gb"] * (1 << 30))
    if args.streams:
        cfg = dict(cfg, streams=args.streams)
    for A, r in list(zip(mats, trace))[: args.warmup]:
        rsvd.solve(A, r["k"], r["p"], r["q"], seed=r["seed"])
    torch.cuda.synchronize()

    def replay(poisson, graphs=True):
        srv = rsvd.Server(dev, hbm_budget_bytes=budget, n_streams=cfg["streams"])
        srv.use_graphs(graphs)
        t0 = time.perf_counter()
        reqs = []
        for A, r in zip(mats, trace):
            if poisson:
                delay = t0 + r["arrival"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            reqs.append(srv.submit(A, r["k"], r["p"], r["q"], seed=r["seed"]))
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        st["graph_launches"], st["graph_instantiations"], st["graph_fallbacks"] = srv.graph_stats()
        srv.close()
        return reqs, st, wall

    reqs_p, st_p, wall_p = replay(True)
    print(f"bench: Poisson replay: {st_p}", file=sys.stderr, flush=True)
    reqs_s, st_s, wall_s = replay(False)
    print(f"bench: saturation replay: {st_s}", file=sys.stderr, flush=True)
    _, st_d, wall_d = replay(False, graphs=False)
    print(f"bench: saturation replay, direct launches: {st_d}", file=sys.stderr, flush=True)
    # Alone-vs-mix: every result of the saturation replay against a solve alone.
    same = 0
    for A, r, rq in zip(mats, trace, reqs_s):
        out = rsvd.solve(A, r["k"], r["p"], r["q"], seed=r["seed"])
        same += int(torch.equal(out["S"], rq.S) and torch.equal(out["U"], rq.U) and torch.equal(out["Vt"], rq.Vt))
    torch.cuda.synchronize()
    flops = sum((2 * r["q"] + 2) * 2.0 * r["m"] * r["n"] * rsvd.l_used(r["m"], r["n"], r["k"], r["p"]) for r in trace)
    out = {
        "metric": METRIC, "value": st_s["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": len(trace),
        "warmup": args.warmup, "ms_per_step": 1e3 / st_s["solves_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c5_serving: {len(trace)} FP32 requests, m,n log-uniform in [256, 8192] "
                               "(half-octave grid), k in {10..128}, p=10, q in {0,1,2}, alternating geometric / "
                               "polynomial spectra; request server with "
                               f"{cfg['streams']} streams and a {cfg['budget_gb']} GiB workspace budget",
                   "requests": len(trace), "offered_rate_per_s": cfg["rate"]},
        "p50_ms": st_p["p50_ms"], "p99_ms": st_p["p99_ms"],
        "poisson_replay": {"achieved_solves_per_s": len(trace) / wall_p, **st_p},
        "saturation_replay": {"wall_s": wall_s, **st_s},
        "saturation_replay_direct_launches": {"wall_s": wall_d, **st_d},
        "tflops_algorithmic_saturation": flops / wall_s / 1e12,
        "alone_equals_mix": f"{same}/{len(trace)}",
        "roofline": None,
    }
    if not args.no_cpu_baseline:
        from oracle.rsvd import rsvd_alg4
        sample = [i for i, r in enumerate(trace) if r["m"] * r["n"] <= 1448 * 1448][:40]
        tc = time.perf_counter()
        errs = []
        for i in sample:
            r = trace[i]
            Ah = mats[i].double().cpu().numpy()
            ref = rsvd_alg4(Ah, r["k"], r["p"], r["q"], seed=r["seed"])
            errs.append(float(np.max(np.abs(reqs_s[i].S.cpu().numpy() - ref["S"])) / ref["S"][0]))
            if time.perf_counter() - tc > 25.0:
                sample = sample[: len(errs)]
                break
        tcpu = time.perf_counter() - tc
        try:
            from threadpoolctl import threadpool_info
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:
            threads = len(os.sched_getaffinity(0))
        out["cpu_baseline"] = {"value": len(errs) / tcpu, "unit": "solves/s", "cores": int(threads),
                               "kind": "oracle", "sample": f"{len(errs)} requests of the trace with m*n <= 1448^2, "
                                                           f"FP64, {tcpu:.1f} s"}
        out["rel_err_vs_fp64_sample"] = {"sigma_normwise_max": max(errs), "requests": len(errs)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2_fp32_8192")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the mixed-precision forms after the default workload")
    ap.add_argument("--no-single-pass", action="store_true",
                    help="skip the single-pass Algorithm 6 timing after the default workload")
    ap.add_argument("--streams", type=int, default=0, help="serving workload: stream slots (0 = the config's)")
    ap.add_argument("--input", choices=("workload", "gaussian"), default="workload",
                    help="gaussian: i.i.d. N(0,1)/sqrt(n) matrix of the same shape, drawn on the device without a "
                         "QR; for hardware-counter runs, where the products' traffic does not depend on the values")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "a multi-GPU row-block sharding is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)

    from paper_2402_17794_amd import workloads

    cfg = workloads.CONFIGS[args.config]
    if cfg.get("serving"):
        # One hardware queue per stream slot (HIP maps streams onto
        # GPU_MAX_HW_QUEUES queues, 4 by default, and kernels of streams that
        # share a queue run one after another).  Set before HIP starts.
        os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(32, args.streams or cfg["streams"])))

    import torch
    from paper_2402_17794_amd import prof_summary, rsvd

    if cfg.get("serving"):
        print(json.dumps(bench_serving(args, cfg, torch, rsvd, workloads)), flush=True)
        return
    m, n, k, p, q = cfg["m"], cfg["n"], cfg["k"], cfg["p"], cfg["q"]
    dtype = torch.float32 if cfg["dtype"] == "f32" else torch.float64
    dev = torch.device("cuda:0")
    print(f"bench: generating {args.config} ...", file=sys.stderr, flush=True)
    tg = time.perf_counter()
    if args.input == "gaussian":
        g = torch.Generator(device=dev)
        g.manual_seed(1)
        A = (torch.randn(m, n, device=dev, dtype=torch.float32, generator=g) / float(n) ** 0.5).to(dtype)
    else:
        A64 = workloads.config_matrix(args.config, device=dev)
        A = A64.to(dtype).contiguous()
        del A64
    torch.cuda.synchronize()
    print(f"bench: input ready in {time.perf_counter() - tg:.1f} s", file=sys.stderr, flush=True)

    # A plain copy of known size (a same-type tensor copy: the runtime's blit
    # kernel), outside the timed region: the reference that scales the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run.
    calib_src = torch.ones(prof_summary.CALIB_BYTES // 4, dtype=torch.int32, device=dev)
    calib_dst = torch.empty_like(calib_src)
    for _ in range(2):
        calib_dst.copy_(calib_src)
    torch.cuda.synchronize()
    del calib_src, calib_dst

    if cfg.get("lowp") and args.input == "workload":
        print(json.dumps(bench_lowp(args, cfg, A, torch, rsvd, workloads)), flush=True)
        return

    solver = rsvd.Solver(A, k, p, q, seed=0)
    l = solver.l
    for _ in range(args.warmup):
        solver()
    torch.cuda.synchronize()

    # Timed region: exactly `steps` solves, bracketed by synchronisation.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        solver()
        evs[i][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    info = int(solver.info.item())
    print(f"bench: {args.steps} solves in {dt * 1e3:.2f} ms", file=sys.stderr, flush=True)

    # Two solves in flight: the same solves alternating between two streams,
    # each with its own workspace (a solve's small SVD runs on one compute
    # unit while the next solve's products use the others).  Reported beside
    # the headline, which is one solve at a time.
    streams2 = [torch.cuda.Stream(dev), torch.cuda.Stream(dev)]
    solvers2 = [rsvd.Solver(A, k, p, q, seed=0, stream=st) for st in streams2]
    torch.cuda.synchronize()
    for i in range(2 * args.warmup):
        solvers2[i % 2]()
    torch.cuda.synchronize()
    t2a = time.perf_counter()
    for i in range(args.steps):
        solvers2[i % 2]()
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t2a
    same2 = all(torch.equal(sv.S, solver.S) and torch.equal(sv.U, solver.U) for sv in solvers2)
    del solvers2, streams2

    # Same solves again with every product with A bracketed by HIP events on
    # the solve's stream: per-launch kernel durations for the roofline.
    rsvd.profile_enable(dev, True)
    for _ in range(args.steps):
        solver()
    torch.cuda.synchronize()
    rsvd.profile_enable(dev, False)
    kinds = {}
    for kind in (0, 1, 2):
        tot, cnt = rsvd.profile_read(dev, kind)
        if cnt:
            kinds[kind] = (tot, cnt)
    st1_tot, st1_cnt = rsvd.profile_read(dev, rsvd.PROFILE_STAGE1)
    jac_tot, jac_cnt = rsvd.profile_read(dev, rsvd.PROFILE_JACOBI)
    sweeps = int(solver.sweeps.item())
    dom = max(kinds, key=lambda kk: kinds[kk][0])
    dom_ms = kinds[dom][0] / kinds[dom][1]
    flops_launch = 2.0 * m * n * l
    achieved = flops_launch / (dom_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[cfg["dtype"]]
    gemm_ms = sum(v[0] for v in kinds.values()) / args.steps
    flops_solve = (2 * q + 2) * 2.0 * m * n * l
    jac_ms = jac_tot / max(1, jac_cnt)

    # The residual ||A - QQ^T A|| (spectral estimate, t = 4, and Frobenius
    # norm), optional in a solve and timed separately: ms per solve with it
    # minus ms per solve without it.
    res_solver = rsvd.Solver(A, k, p, q, seed=0, residual=3, residual_iters=4)
    res_solver()
    torch.cuda.synchronize()
    nres = max(3, args.steps // 4)
    tr0 = time.perf_counter()
    for _ in range(nres):
        res_solver()
    torch.cuda.synchronize()
    res_ms = (time.perf_counter() - tr0) / nres * 1e3 - dt / args.steps * 1e3
    res_gpu = res_solver.res.cpu().numpy()
    del res_solver

    # HBM bytes per launch of the dominant kernel from the committed counter
    # summary, only while the GEMM sources are the ones the counters measured.
    traffic = None
    tr = prof_summary.read_traffic(os.path.join(ROOT, "profiles", f"gemm_tn_{args.config}_traffic.txt"))
    if tr is not None and dom == 2 and tr[1] == prof_summary.gemm_source_hash():
        traffic = tr[0]

    S_gpu = solver.S.cpu().numpy()
    out = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfg["dtype"],
        "data": "synthetic",
        "config": {"workload": _describe(args.config, cfg) if args.input == "workload" else
                   f"{args.config} shape with a Gaussian N(0,1/n) matrix (counter runs)",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "l": l},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "tflops_algorithmic": flops_solve / (dt / args.steps) / 1e12,
        "gemm_ms_per_solve": gemm_ms,
        # The range finder as a whole (Stage 1: sketch, q power iterations and
        # every orthonormalisation), (2q + 1) 2 m n l flops over its event time.
        "range_finder": {"ms": st1_tot / max(1, st1_cnt),
                         "tflops": (2 * q + 1) * 2.0 * m * n * l / (st1_tot / max(1, st1_cnt) * 1e-3) / 1e12,
                         "frac_of_peak": (2 * q + 1) * 2.0 * m * n * l / (st1_tot / max(1, st1_cnt) * 1e-3) / 1e12
                         / PEAK_TFLOPS[cfg["dtype"]]},
        "info": info,
        "residual": {"spectral_estimate_t4": float(res_gpu[0]), "frobenius": float(res_gpu[1]),
                     "ms_per_solve": res_ms},
        "roofline_contraction": {
            "bound": "mfma",
            "kernel": KIND_NAMES[dom].replace("float", "double") if cfg["dtype"] == "f64" else KIND_NAMES[dom],
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": float(m * n * A.element_size()),
            "avg_launch_ms": dom_ms,
            "flops_per_launch": flops_launch,
            "launches_per_solve": kinds[dom][1] / args.steps,
            "ms_per_solve": kinds[dom][0] / args.steps,
        },
        "small_svd_jacobi": {"ms": jac_ms, "sweeps": sweeps, "l": l},
        "two_in_flight": {"solves_per_s": args.steps / dt2, "ms_per_solve": dt2 / args.steps * 1e3,
                          "results_equal_single_stream": bool(same2),
                          "note": "the same solves alternating between two streams with separate workspaces"},
    }
    # The roofline of the kernel that takes the most time per solve: the
    # product kind above, or the small SVD's Jacobi iteration (FP64 vector
    # work on one compute unit, against the FP64 vector peak).
    jflops = _jacobi_flops(l, sweeps)
    if jac_ms > kinds[dom][0] / args.steps:
        ja = jflops / (jac_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "small SVD one-sided Jacobi (jacobi_oe_kernel<R> / jacobi_blk_*)",
                           "achieved": ja, "peak": PEAK_VALU_TFLOPS["f64"], "unit": "TFLOP/s",
                           "frac": ja / PEAK_VALU_TFLOPS["f64"], "traffic": None, "avg_launch_ms": jac_ms,
                           "flops_per_launch": jflops, "launches_per_solve": 1.0,
                           "note": "Jacobi span of one solve; flops = sweeps * l(l-1)/2 * 6 l"}
    else:
        out["roofline"] = dict(out["roofline_contraction"])

    if not args.no_cpu_baseline and args.input == "workload":
        from oracle.rsvd import rsvd_alg4
        threads = _blas_threads()
        Ah = A.double().cpu().numpy()
        print("bench: running the FP64 CPU oracle on the same matrix ...", file=sys.stderr, flush=True)
        # Whole solves of the same workload until about 10 s of CPU work (at most 5).
        tc = time.perf_counter()
        nsol = 0
        while True:
            ref = rsvd_alg4(Ah, k, p, q, seed=0)
            nsol += 1
            tcpu = time.perf_counter() - tc
            if tcpu >= 10.0 or nsol >= 5:
                break
        out["cpu_baseline"] = {"value": nsol / tcpu, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
                               "sample": f"{nsol} full solve(s) of the same workload ({m}x{n}, k={k}, p={p}, "
                                         f"q={q}) in float64, {tcpu:.1f} s wall clock incl. Omega generation",
                               "cpu_model": _cpu_model()}
        if m * n <= 2048 * 2048:
            st_rate, st_n = _oracle_single_thread(Ah, k, p, q)
            out["cpu_baseline"]["single_thread"] = {"value": st_rate, "unit": "solves/s", "solves": st_n}
        S_ref = ref["S"]
        from oracle.rsvd import spectral_norm_power
        E = Ah - ref["Q"] @ (ref["Q"].T @ Ah)
        out["residual"]["oracle_spectral_estimate_t4"] = spectral_norm_power(E, iters=4, block=16, seed=0)
        out["residual"]["oracle_frobenius"] = float(np.linalg.norm(E))
        del E
        out["rel_err_vs_fp64"] = {
            "sigma_normwise_max": float(np.max(np.abs(S_gpu - S_ref)) / S_ref[0]),
            "sigma_relative_max": float(np.max(np.abs(S_gpu - S_ref) / S_ref)),
        }
    sig = workloads.config_sigma(args.config)
    if sig is not None and args.input == "workload":
        out["err_vs_true_spectrum_normwise"] = float(np.max(np.abs(S_gpu - sig[:k])) / sig[0])
    if args.config == "c2_fp32_8192" and not args.no_single_pass:
        print("bench: single-pass Algorithm 6 on the same matrix ...", file=sys.stderr, flush=True)
        out["single_pass"] = bench_single_pass(args, A, cfg, torch, rsvd, prof_summary,
                                               not args.no_cpu_baseline and args.input == "workload")
    if args.config == "c2_fp32_8192" and args.input == "workload" and not args.no_c4:
        # The largest configuration, timed in the same run: the mixed-precision
        # workload in its three storage forms (5 timed solves each, no oracle
        # leg here; its errors against the FP64 oracle come from
        # `--config c4_mixed_32768x16384`).
        del solver, A
        torch.cuda.empty_cache()
        c4 = "c4_mixed_32768x16384"
        print(f"bench: generating {c4} ...", file=sys.stderr, flush=True)
        A4 = workloads.config_matrix(c4, device=dev).float().contiguous()
        torch.cuda.synchronize()
        a4 = argparse.Namespace(steps=5, warmup=2, no_cpu_baseline=True, config=c4)
        r4 = bench_lowp(a4, workloads.CONFIGS[c4], A4, torch, rsvd, workloads)
        out[c4] = {"workload": r4["config"]["workload"], "forms": r4["forms"]}
        del A4
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

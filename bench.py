#!/usr/bin/env python3
"""Forward-solver benchmark of the Bernstein-Bezier DG path on one MI355X.

Headline workload (the forward-throughput configuration): the unit cube split
into 16^3 x 6 = 24,576 affine tets with interior vertices jittered by +-10% of
h (seeded), order N = 5 (Np = 56), fields p,u,v,w, unit wavespeed, rigid
walls, standing-mode initial pressure, LSRK4 with dt = 0.5 h/(N+1)^2.
A bench "step" is one LSRK4 time step = five fused stage kernels (volume +
surface + update each); inputs are resident in HBM before timing starts.

Timing: W warm-up steps, then more warm-up runs until at least 200 ms of
wall-clock time has passed, then 5 timed runs of K steps each, every run
bracketed by torch.cuda.synchronize() and HIP events recorded on the stream
the kernels run on; the reported time is the median run.

Prints one JSON line: DoF-stage updates/s (4 K Np per stage) for FP64 (the
headline value), the FP32 run on the same workload, the two dense nodal
comparators (MFMA, and element per thread), the order sweep on 32^3 x 6 = 196,608 tets (the configuration
whose fields do not fit in the 256 MB last-level cache, where the stage
kernel's roofline placement is taken), the 64-shot batched workload, the
misfit gradient, a streaming-copy probe, and the FP64 CPU oracle timed on
bounded samples on the host cores.
"""
import argparse
import gc
import json
import os
import statistics
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
ROOT = os.path.dirname(os.path.abspath(__file__))
REPS = 5
MIN_WARM_MS = 200.0
LEGS = ("c2", "fp32", "nodal", "c3", "batched", "gradient", "copy", "cpu")


def recorded_traffic(kernel, workload):
    """Calibrated FETCH_SIZE + WRITE_SIZE bytes per dispatch recorded under
    profiles/ for this kernel and workload, if the kernel sources have not
    changed since the counters were taken (else None)."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "stage_traffic.json")) as f:
            entries = json.load(f)["entries"]
    except (OSError, ValueError, KeyError):
        return None
    for e in entries:
        if e.get("kernel") != kernel or not e.get("workload", "").startswith(workload):
            continue
        h = hashlib.sha256()
        try:
            for src in e["sources"]:
                with open(os.path.join(ROOT, src), "rb") as f:
                    h.update(f.read())
        except OSError:
            continue
        if h.hexdigest() == e.get("source_sha256"):
            return e["bytes_per_dispatch"]
    return None


def stage_kernel_name(N, dtype, nt):
    """Name of the stage kernel instantiation the library launches for order
    N: waves per workgroup (three at N = 8 in FP64, else four) and whether
    the non-temporal-store variant runs (reported by the library)."""
    t = "double" if dtype == "f64" else "float"
    wpb = 3 if (N == 8 and dtype == "f64") else 4
    return "bb_stage_kernel<%d, %s, 0, %d, %s>" % (N, t, wpb, "true" if nt else "false")


def algorithmic_bytes_per_element(N, word):
    """Bytes a fused stage must move per element, averaged over the five
    stages of an LSRK4 step: read q (4 Np words) and the residual (4 Np,
    skipped by the first stage, whose residual coefficient is zero), read
    the four faces' neighbour traces (16 Nfp), write q and the residual
    (8 Np); 14 words of geometry and 20 B of connectivity.
    = w (16 Np + 16 Nfp + 14) + 20 - w 4 Np / 5."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nfp = (N + 1) * (N + 2) // 2
    return word * (16 * Np + 16 * Nfp + 14) + 20 - word * 4.0 * Np / 5.0


def timed_runs(torch, run, stream):
    """Wall-clock warm-up of at least MIN_WARM_MS (run() repeated, each
    followed by a device synchronisation), then REPS timed runs, each
    bracketed by synchronisations and by HIP events on `stream`.  Returns
    the list of run times in ms."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < MIN_WARM_MS:
        run()
        torch.cuda.synchronize()
    out = []
    for _ in range(REPS):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        run()
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def time_solver(P, torch, N, mesh, c, q0, dt, steps, warmup, dtype, basis="bb"):
    """Median ms of REPS runs of `steps` LSRK4 steps (after W warm-up steps
    and the wall-clock warm-up); also the run times, whether the state
    stayed finite, the state after the W warm-up steps plus one timed-size
    run (for error comparisons), and whether non-temporal stores ran."""
    s = P.Solver(N, mesh, c, dtype=dtype, basis=basis)
    q = torch.from_numpy(q0).to("cuda", s.torch_dtype)
    stream = torch.cuda.current_stream()
    if warmup:
        s.run(q, dt, warmup, stream=stream)
    s.run(q, dt, steps, stream=stream)
    torch.cuda.synchronize()
    q_ref = q.clone()
    ms = timed_runs(torch, lambda: s.run(q, dt, steps, stream=stream), stream)
    finite = bool(torch.isfinite(q).all().item())
    nt = basis == "bb" and s.nontemporal_stores()
    s.close()
    del q
    return statistics.median(ms), ms, finite, q_ref, nt


def roofline_obj(N, dtype, K, stage_us, nt, workload_tag, cache_assisted):
    w = 8 if dtype == "f64" else 4
    bytes_launch = algorithmic_bytes_per_element(N, w) * K
    achieved = bytes_launch / (stage_us * 1e-6) / 1e9
    kern = stage_kernel_name(N, dtype, nt)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(kern, workload_tag),
            "kernel": kern, "workload": workload_tag, "bytes_per_launch": bytes_launch,
            "bytes_per_element": algorithmic_bytes_per_element(N, w), "avg_launch_us": stage_us,
            "cache_assisted": cache_assisted}


def nodal_entry(kind, N, dtype, K, stage_us, finite):
    """Throughput of a dense nodal comparator stage: the MFMA kernel ("nodal",
    24 Np^2 + 32 Np Nfp FLOP per element: three derivative matrices on four
    fields and the four-face lift, against the dense MFMA peak of its type) or
    the element-per-thread kernel ("nodal_ept", which applies the derivative
    matrices to p and to the three h_d = grad(lambda_d).u only, 12 Np^2 + 32
    Np Nfp FLOP, against the vector FMA peak of its type)."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nfp = (N + 1) * (N + 2) // 2
    if kind == "nodal":
        flop = K * (24 * Np * Np + 32 * Np * Nfp)
        peak_key, peak = "mfma_peak_tflops", (78.6 if dtype == "f64" else 157.3)
    else:
        flop = K * (12 * Np * Np + 32 * Np * Nfp)
        peak_key, peak = "vector_peak_tflops", (78.6 if dtype == "f64" else 157.3)
    tf = flop / (stage_us * 1e-6) / 1e12
    return {"stage_us": stage_us, "tflops": tf, peak_key: peak, "peak_frac": tf / peak, "finite": finite,
            "dof_stage_per_s": 4.0 * K * Np / (stage_us * 1e-6)}


def time_c3(P, torch, workload, ic, orders, dtypes, steps, nodal_steps, warmup):
    """Order sweep on 32^3 x 6 = 196,608 tets, c ~ U[1,3], Gaussian pulse:
    per-stage time and HBM roofline placement of the BB stage for each
    order and element type, and the dense nodal comparator beside it."""
    cfg, VX, EToV, c = workload.build_preset("c3")
    K = cfg["K"]
    mesh = P.mesh_geometry(VX, EToV)
    out = {"workload": "unit cube 32^3x6 = %d tets, c~U[1,3] (seeded), Gaussian pulse IC, rigid walls, "
                       "dt = 0.5 h/(3 (N+1)^2); %d steps per timed run (median of %d), nodal %d"
                       % (K, steps, REPS, nodal_steps), "K": K, "orders": {}}
    for N in orders:
        pre = workload.preset("c3", N=N)
        dt = pre["dt"]
        Np = pre["Np"]
        q0 = ic.initial_state(N, VX, EToV, workload.INITIAL_FIELDS[cfg["ic"]])
        row = {}
        for dtype in dtypes:
            med, runs, ok, _, nt = time_solver(P, torch, N, mesh, c, q0, dt, steps, warmup, dtype)
            st = med * 1e3 / (5 * steps)
            r = roofline_obj(N, dtype, K, st, nt, "c3 N=%d %s" % (N, dtype), False)
            r.update(stage_us_runs=[m * 1e3 / (5 * steps) for m in runs], finite=ok,
                     dof_stage_per_s=4.0 * K * Np / (st * 1e-6))
            row[dtype] = r
        if nodal_steps > 0:
            x0 = ic.initial_state(N, VX, EToV, workload.INITIAL_FIELDS[cfg["ic"]], basis="nodal")
            for dtype in dtypes:
                for kind in ("nodal", "nodal_ept"):
                    med, runs, ok, _, _ = time_solver(P, torch, N, mesh, c, x0, dt, nodal_steps, 0, dtype,
                                                      basis=kind)
                    st = med * 1e3 / (5 * nodal_steps)
                    e = nodal_entry(kind, N, dtype, K, st, ok)
                    e["bb_speedup"] = st / row[dtype]["avg_launch_us"]
                    row[kind + "_" + dtype] = e
        out["orders"][str(N)] = row
        gc.collect()
    return out


def time_batched(P, torch, workload, steps):
    """64 shots with Ricker point sources on 24,576 tets, N = 4, FP32: the
    5 * steps stages in persistent launches of up to 1024 steps each (one
    launch for the default 500 steps; launch shape autotuned)."""
    cfg, VX, EToV, c = workload.build_preset("c4")
    N, K, Np, S, dt = cfg["N"], cfg["K"], cfg["Np"], cfg["shots"], cfg["dt"]
    mesh = P.mesh_geometry(VX, EToV)
    bs = P.BatchedSolver(N, mesh, c, S, sources=workload.source_positions(S), receivers=workload.receiver_grid(),
                         f0=cfg["f0"], ts=cfg["ts"], dtype="f32")
    wpb = bs.tune()
    stream = torch.cuda.current_stream()
    q = bs.empty_state()
    bs.run(q, dt, 2, stream=stream)  # warm-up launch
    q.zero_()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    tr = bs.run(q, dt, steps, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    bs.check()
    stages = 5 * steps
    stage_us = ms * 1e3 / stages
    gbs = algorithmic_bytes_per_element(N, 4) * K * S / (stage_us * 1e-6) / 1e9
    finite = bool(torch.isfinite(q).all().item() and torch.isfinite(tr).all().item())
    bs.close()
    del q
    # the same run in FP64 (untimed) for the FP32 error of the traces
    b64 = P.BatchedSolver(N, mesh, c, S, sources=workload.source_positions(S), receivers=workload.receiver_grid(),
                          f0=cfg["f0"], ts=cfg["ts"], dtype="f64", wpb=4)
    tr64 = b64.run(b64.empty_state(), dt, steps)
    b64.check()
    err32 = float(torch.linalg.norm(tr.double() - tr64) / torch.linalg.norm(tr64))
    b64.close()
    return {"workload": "%d shots, Ricker f0=%g, %d receivers, unit cube %d^3x6 = %d tets, N=%d, c~U[%g,%g], "
                        "FP32, %d steps in %d persistent launch(es)" % (S, cfg["f0"], 64, cfg["n"], K, N,
                                                                         cfg["c"][0], cfg["c"][1], steps,
                                                                         (steps + 1023) // 1024),
            "value": 4.0 * K * Np * S * stages / (ms * 1e-3), "unit": "DoF-stage/s", "ms_total": ms,
            "stage_us": stage_us, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS, "waves_per_workgroup": wpb,
            "finite": finite, "traces_rel_l2_error_vs_fp64": err32}


def time_gradient(P, torch, workload, steps):
    """Misfit and its gradient in m = c^2: 8 shots on 24,576 tets, N = 5,
    FP32 states (FP64 gradient sums), observations from the FP64 forward run
    at a blob model, gradient at m = 1, checkpoints every 50 steps, stage
    records of as many segments as the free device memory holds.  The ratio
    is (J + dJ/dm) over a plain forward run of the same shots (traces only,
    no checkpoints or records)."""
    cfg, VX, EToV, _ = workload.build_preset("c5")
    N, K, S, dt = cfg["N"], cfg["K"], cfg["shots"], cfg["dt"]
    mesh = P.mesh_geometry(VX, EToV)
    src, rec = workload.plane_sources(S), workload.receiver_grid()
    m_true = workload.blob_model(VX, EToV)
    # observations: FP64 forward at m_true
    obs_run = P.BatchedSolver(N, mesh, np.sqrt(m_true), S, sources=src, receivers=rec, f0=cfg["f0"], ts=cfg["ts"],
                              dtype="f64", wpb=4)
    d_obs = obs_run.run(obs_run.empty_state(), dt, steps).clone()
    obs_run.close()
    del obs_run
    gc.collect()
    torch.cuda.empty_cache()
    mf = P.Misfit(N, mesh, np.ones(K), S, src, rec, d_obs, dt, steps, f0=cfg["f0"], ts=cfg["ts"],
                  ckpt_every=cfg["ckpt_every"], dtype="f32", rec_segments="max")
    mf.evaluate()
    mf.gradient()  # warm-up
    q_plain = mf.batched.empty_state()
    mf.batched.run(q_plain, dt, steps)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ev[0].record(stream)
    mf.batched.run(q_plain.zero_(), dt, steps)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ev[2].record(stream)
    J = mf.evaluate()
    ev[3].record(stream)
    g = mf.gradient()
    ev[4].record(stream)
    torch.cuda.synchronize()
    mf.check()
    t_plain, t_fwd, t_adj = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3]), ev[3].elapsed_time(ev[4])
    finite = bool(torch.isfinite(g).all().item())
    g = g.clone()
    M = mf.rec_segments
    mf.close()
    del mf, q_plain
    gc.collect()
    torch.cuda.empty_cache()
    # the same gradient with FP64 states (untimed) for the FP32 error
    m64 = P.Misfit(N, mesh, np.ones(K), S, src, rec, d_obs, dt, steps, f0=cfg["f0"], ts=cfg["ts"],
                   ckpt_every=cfg["ckpt_every"], dtype="f64")
    J64 = float(m64.evaluate().item())
    g64 = m64.gradient()
    m64.check()
    m64.close()
    del m64
    gc.collect()
    out = {"workload": "misfit gradient dJ/dm, %d shots (Ricker f0=%g on z=0.9), 64 receivers, %d^3x6 = %d tets, "
                       "N=%d, FP32 states / FP64 sums, %d steps, checkpoints every %d, records of %d segments" % (
                           S, cfg["f0"], cfg["n"], K, N, steps, cfg["ckpt_every"], M),
           "J": float(J.item()), "plain_forward_ms": t_plain, "forward_ms": t_fwd, "reverse_ms": t_adj,
           "rec_segments": M, "grad_over_forward": (t_fwd + t_adj) / t_plain, "reverse_over_forward": t_adj / t_plain,
           "finite": finite, "J_rel_error_vs_fp64": abs(float(J.item()) - J64) / abs(J64),
           "grad_rel_l2_error_vs_fp64": float(torch.linalg.norm(g - g64) / torch.linalg.norm(g64))}
    return out


def copy_probe(torch, nbytes=1 << 30, reps=20):
    """Bandwidth of a plain streaming copy (read + write bytes per second)."""
    from paper_1512_06025_amd import _lib
    lib = _lib.load()
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sp = _lib.ctypes.c_void_p(stream.cuda_stream)
    _lib.check(lib.bbdg_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, sp), "bbdg_copy_probe")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lib.bbdg_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, sp)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(src, dst))
    del src, dst
    return {"bytes_moved": 2 * nbytes, "us": ms * 1e3, "GBs": 2 * nbytes / (ms * 1e-3) / 1e9, "ok": ok}


def host_description():
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count(), "cpu": cpu}


def cpu_baseline(workload, ic_c2, gpu_stage_us):
    """The FP64 oracle (NumPy, dense operators) timed on the host cores on
    bounded samples: one LSRK4 step of the headline workload with all BLAS
    threads (the reported value) and one of its stages on a single thread;
    the whole 10-step run of the 384-tet N = 3 workload; one stage of the
    196,608-tet order sweep for N = 1, 3, 5.  Per-stage times beside the
    GPU's.  The oracle is test infrastructure: this is a reported baseline,
    not a fallback."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import dg
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    per_stage = {}
    # headline workload: one LSRK4 step (5 stages), all threads
    cfg, VX, EToV, c = workload.build_preset("c2")
    prob = dg.Problem(VX, EToV, cfg["N"], c)
    K, Np = prob.K, prob.Np
    if ic_c2 is None:
        ic_c2 = dg.initial_state(prob, workload.standing_mode_p0)
    t0 = time.perf_counter()
    q = prob.lsrk4(ic_c2, cfg["dt"], 1)
    sec = time.perf_counter() - t0
    per_stage["c2"] = sec / 5
    # the same workload, one stage on one thread
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = prob.rhs(q)
        q = q + cfg["dt"] * r
        per_stage_1t = time.perf_counter() - t0
    del prob, q, r
    # 384 tets, N = 3: the whole 10-step run
    cfg1, VX1, EToV1, c1 = workload.build_preset("c1")
    p1 = dg.Problem(VX1, EToV1, cfg1["N"], c1)
    q1 = dg.initial_state(p1, workload.standing_mode_p0)
    t0 = time.perf_counter()
    p1.lsrk4(q1, cfg1["dt"], cfg1["steps"])
    per_stage["c1"] = (time.perf_counter() - t0) / (5 * cfg1["steps"])
    # order sweep mesh, N = 1, 3, 5: one stage (right-hand side + update) each
    cfg3, VX3, EToV3, c3 = workload.build_preset("c3")
    for N in (1, 3, 5):
        p3 = dg.Problem(VX3, EToV3, N, c3)
        q3 = workload.random_coeffs(p3.K, p3.Np, seed=90 + N)
        t0 = time.perf_counter()
        r3 = p3.rhs(q3)
        q3 = q3 + workload.preset("c3", N=N)["dt"] * r3
        per_stage["c3_N%d" % N] = time.perf_counter() - t0
        del p3, q3, r3
        gc.collect()
    return {
        "value": 4.0 * K * Np / per_stage["c2"],
        "unit": "DoF-stage/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "FP64 dense-operator NumPy oracle: 1 LSRK4 step (5 stages) of the headline workload "
                  "(K=%d, N=%d) with %d BLAS threads (NumPy's elementwise and einsum parts run on one "
                  "thread) = value; plus one single-thread stage of the same workload, the whole 10-step "
                  "384-tet N=3 run, and one stage of the 196,608-tet mesh for N=1,3,5" % (K, cfg["N"], threads),
        "host": host_description(),
        "single_thread_value": 4.0 * K * Np / per_stage_1t,
        "oracle_stage_s": per_stage,
        "gpu_stage_s": gpu_stage_us,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", help="named workload of the headline leg (c1..c3)")
    ap.add_argument("--order", type=int, default=None, help="override N of the headline leg")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated subset of %s" % ",".join(LEGS))
    ap.add_argument("--c3-orders", default="5,7,9")
    ap.add_argument("--c3-dtypes", default="f64,f32")
    ap.add_argument("--c3-steps", type=int, default=40, help="LSRK4 steps per timed run of the order sweep")
    ap.add_argument("--c3-nodal-steps", type=int, default=2, help="0 skips the nodal comparator on the sweep")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--gradient-steps", type=int, default=500)
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="only run the streaming-copy probe (counter calibration)")
    for leg in LEGS:
        ap.add_argument("--no-" + ("cpu-baseline" if leg == "cpu" else "copy-probe" if leg == "copy" else leg),
                        dest="skip_" + leg, action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on a single GPU; multi-GPU runs (--gpus %d) are not "
              "supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x) - set(l for l in LEGS if getattr(args, "skip_" + l))

    import torch

    import paper_1512_06025_amd as P
    import workload
    from paper_1512_06025_amd import ic

    if args.copy_probe_only:
        print(json.dumps({"copy_probe": copy_probe(torch)}), flush=True)
        return

    over = {} if args.order is None else {"N": args.order}
    cfg, VX, EToV, c = workload.build_preset(args.config, **over)
    N, K, Np, dt = cfg["N"], cfg["K"], cfg["Np"], cfg["dt"]
    Nfp = (N + 1) * (N + 2) // 2
    mesh = P.mesh_geometry(VX, EToV)
    q0 = ic.initial_state(N, VX, EToV, workload.INITIAL_FIELDS[cfg["ic"]])

    stages = 5 * args.steps
    dof = 4.0 * K * Np
    out = {
        "metric": "DoF-stage updates/s & % HBM roofline (BB vs nodal, FP64/FP32); grad/forward x",
        "value": None,
        "unit": "DoF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "BB-DG acoustic forward, unit cube %d^3x6 = %d tets%s, N=%d (Np=%d), %s IC, "
                        "rigid walls, LSRK4 dt=%.6g, %d steps per timed run" % (
                            cfg["n"], K, ", interior vertices jittered +-%g h" % cfg["jitter"] if cfg["jitter"] else "",
                            N, Np, cfg["ic"], dt, args.steps),
            "K": K, "N": N, "Np": Np, "Nfp": Nfp, "stages": stages,
            "parallelism": "single GPU",
        },
        "timing": "W warm-up steps, >= %g ms wall-clock warm-up, then the median of %d timed runs of K steps "
                  "(HIP events on the kernels' stream, device synchronised around each run)" % (MIN_WARM_MS, REPS),
    }
    gpu_stage_s = {}
    q64 = None
    ms64 = None
    if "c2" in legs:
        ms64, runs64, ok64, q64, nt64 = time_solver(P, torch, N, mesh, c, q0, dt, args.steps, args.warmup, "f64")
        stage_us = ms64 * 1e3 / stages
        out["value"] = dof * stages / (ms64 * 1e-3)
        out["ms_per_step"] = ms64 / args.steps
        out["ms_per_step_runs"] = [m / args.steps for m in runs64]
        out["stage_us"] = stage_us
        out["finite"] = ok64
        gpu_stage_s[args.config] = stage_us * 1e-6
        # at 24,576 tets the fields (88 MB per copy) fit in the 256 MB last-level cache
        out["c2_roofline"] = roofline_obj(N, "f64", K, stage_us, nt64, args.config,
                                          cache_assisted=bool(K * Np * 4 * 8 * 3 <= 256 * 1024 * 1024))
    if "fp32" in legs:
        ms32, runs32, ok32, q32, _ = time_solver(P, torch, N, mesh, c, q0, dt, args.steps, args.warmup, "f32")
        st32 = ms32 * 1e3 / stages
        a32 = algorithmic_bytes_per_element(N, 4) * K / (st32 * 1e-6) / 1e9
        f32 = {"value": dof * stages / (ms32 * 1e-3), "ms_per_step": ms32 / args.steps,
               "stage_us": st32, "achieved_GBs": a32, "frac": a32 / HBM_PEAK_GBS, "finite": ok32}
        if q64 is not None:
            # both runs took the same W + K steps from q0 before the copy;
            # the FP64 path matches the oracle to 1e-12
            f32["rel_l2_error_vs_fp64"] = float(torch.linalg.norm(q32.double() - q64) / torch.linalg.norm(q64))
        out["fp32"] = f32
        del q32
    if "nodal" in legs:
        x0 = ic.initial_state(N, VX, EToV, workload.INITIAL_FIELDS[cfg["ic"]], basis="nodal")
        nod = {}
        for kind in ("nodal", "nodal_ept"):
            for dtn in ("f64", "f32"):
                msn, runsn, okn, _, _ = time_solver(P, torch, N, mesh, c, x0, dt, args.steps, args.warmup, dtn,
                                                    basis=kind)
                e = nodal_entry(kind, N, dtn, K, msn * 1e3 / stages, okn)
                e["value"] = dof * stages / (msn * 1e-3)
                bb = ms64 if dtn == "f64" else out.get("fp32", {}).get("ms_per_step", 0) * args.steps
                if bb:
                    e["bb_speedup"] = msn / bb
                nod[dtn if kind == "nodal" else "ept_" + dtn] = e
        out["nodal"] = nod
    del q64
    if "c3" in legs:
        orders = [int(x) for x in args.c3_orders.split(",") if x]
        dtypes = [x for x in args.c3_dtypes.split(",") if x]
        c3 = time_c3(P, torch, workload, ic, orders, dtypes, args.c3_steps, args.c3_nodal_steps, args.warmup)
        out["c3"] = c3
        for Nk, row in c3["orders"].items():
            if "f64" in row:
                gpu_stage_s["c3_N%s" % Nk] = row["f64"]["avg_launch_us"] * 1e-6
        head = c3["orders"].get("5", c3["orders"].get(str(orders[0]), {}))
        if "f64" in head:
            out["roofline"] = head["f64"]
    if "roofline" not in out and "c2_roofline" in out:
        out["roofline"] = out["c2_roofline"]
    if "batched" in legs:
        out["batched"] = time_batched(P, torch, workload, args.batched_steps)
    if "gradient" in legs:
        out["gradient"] = time_gradient(P, torch, workload, args.gradient_steps)
    if "copy" in legs:
        cp = copy_probe(torch)
        for key in ("roofline", "c2_roofline"):
            if key in out:
                out[key]["copy_probe_GBs"] = cp["GBs"]
                out[key]["frac_of_copy_probe"] = out[key]["achieved"] / cp["GBs"]
    # every device buffer is released before the host-only baseline and the exit
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if "cpu" in legs:
        if "c1" not in gpu_stage_s and "c2" in legs:
            cfg1, VX1, EToV1, c1 = workload.build_preset("c1")
            x1 = ic.initial_state(cfg1["N"], VX1, EToV1, workload.INITIAL_FIELDS[cfg1["ic"]])
            m1, _, _, _, _ = time_solver(P, torch, cfg1["N"], P.mesh_geometry(VX1, EToV1), c1, x1, cfg1["dt"],
                                         cfg1["steps"], 0, "f64")
            gpu_stage_s["c1"] = m1 * 1e-3 / (5 * cfg1["steps"])
        headline_is_c2 = args.config == "c2" and args.order is None
        # the oracle takes (4, K, Np) states; q0 is in the solver's element-major (K, 4, Np)
        q0_oracle = np.ascontiguousarray(np.swapaxes(q0, 0, 1)) if headline_is_c2 else None
        out["cpu_baseline"] = cpu_baseline(workload, q0_oracle, gpu_stage_s)
    print(json.dumps(out), flush=True)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Forward-solver benchmark of the Bernstein-Bezier DG path on one MI355X.

Default workload (the forward-throughput configuration): the unit cube split
into 16^3 x 6 = 24,576 affine tets with interior vertices jittered by +-10% of
h (seeded), order N = 5 (Np = 56), fields p,u,v,w, unit wavespeed, rigid
walls, standing-mode initial pressure, LSRK4 with dt = 0.5 h/(N+1)^2.
A bench "step" is one LSRK4 time step = five fused stage kernels (volume +
surface + update each); inputs are resident in HBM before timing starts.

Prints one JSON line: DoF-stage updates/s (4 K Np per stage) for FP64 (the
headline value), plus the FP32 run on the same workload, the roofline
placement of the stage kernel, and the FP64 CPU oracle timed on a bounded
sample on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
ROOT = os.path.dirname(os.path.abspath(__file__))


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


def stage_kernel_name(N, K):
    """Name of the FP64 stage kernel instantiation the library launches for
    order N on K elements: waves per workgroup (three at N = 8, else four)
    and non-temporal output stores when the state, residual and second
    buffer (3 x 4 K Np doubles) exceed the 256 MB last-level cache."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    wpb = 3 if N == 8 else 4
    nt = 3 * 4 * K * Np * 8 > 256 * 1024 * 1024
    return "bb_stage_kernel<%d, double, 0, %d, %s>" % (N, wpb, "true" if nt else "false")


def algorithmic_bytes_per_element(N, word):
    """w (16 Np + 16 Nfp + 14) + 20 bytes: read q and res, read the 4 faces'
    neighbour traces, write q and res; 14 words of geometry, 20 B of indices."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nfp = (N + 1) * (N + 2) // 2
    return word * (16 * Np + 16 * Nfp + 14) + 20


def time_gpu(P, torch, N, mesh, c, q0, dt, steps, warmup, dtype, basis="bb"):
    s = P.Solver(N, mesh, c, dtype=dtype, basis=basis)
    q = torch.from_numpy(q0).to("cuda", s.torch_dtype)
    stream = torch.cuda.current_stream()
    if warmup:
        s.run(q, dt, warmup, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.run(q, dt, steps, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    finite = bool(torch.isfinite(q).all().item())
    s.close()
    return ms, finite, q


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
    stages = 5 * steps
    stage_us = ms * 1e3 / stages
    gbs = algorithmic_bytes_per_element(N, 4) * K * S / (stage_us * 1e-6) / 1e9
    finite = bool(torch.isfinite(q).all().item() and torch.isfinite(tr).all().item())
    bs.close()
    # the same run in FP64 (untimed) for the FP32 error of the traces
    b64 = P.BatchedSolver(N, mesh, c, S, sources=workload.source_positions(S), receivers=workload.receiver_grid(),
                          f0=cfg["f0"], ts=cfg["ts"], dtype="f64", wpb=4)
    tr64 = b64.run(b64.empty_state(), dt, steps)
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
    at a blob model, gradient at m = 1, checkpoints every 50 steps."""
    cfg, VX, EToV, _ = workload.build_preset("c5")
    N, K, S, dt = cfg["N"], cfg["K"], cfg["shots"], cfg["dt"]
    mesh = P.mesh_geometry(VX, EToV)
    src, rec = workload.plane_sources(S), workload.receiver_grid()
    m_true = workload.blob_model(VX, EToV)
    # observations: FP64 forward at m_true
    obs_run = P.BatchedSolver(N, mesh, np.sqrt(m_true), S, sources=src, receivers=rec, f0=cfg["f0"], ts=cfg["ts"],
                              dtype="f64", wpb=4)
    d_obs = obs_run.run(obs_run.empty_state(), dt, steps)
    obs_run.close()
    mf = P.Misfit(N, mesh, np.ones(K), S, src, rec, d_obs, dt, steps, f0=cfg["f0"], ts=cfg["ts"],
                  ckpt_every=cfg["ckpt_every"], dtype="f32")
    mf.evaluate()
    mf.gradient()  # warm-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    J = mf.evaluate()
    ev[1].record(stream)
    g = mf.gradient()
    ev[2].record(stream)
    torch.cuda.synchronize()
    t_fwd, t_adj = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    finite = bool(torch.isfinite(g).all().item())
    g = g.clone()
    mf.close()
    # the same gradient with FP64 states (untimed) for the FP32 error
    m64 = P.Misfit(N, mesh, np.ones(K), S, src, rec, d_obs, dt, steps, f0=cfg["f0"], ts=cfg["ts"],
                   ckpt_every=cfg["ckpt_every"], dtype="f64")
    J64 = float(m64.evaluate().item())
    g64 = m64.gradient()
    m64.close()
    out = {"workload": "misfit gradient dJ/dm, %d shots (Ricker f0=%g on z=0.9), 64 receivers, %d^3x6 = %d tets, "
                       "N=%d, FP32 states / FP64 sums, %d steps, checkpoints every %d" % (
                           S, cfg["f0"], cfg["n"], K, N, steps, cfg["ckpt_every"]),
           "J": float(J.item()), "forward_ms": t_fwd, "reverse_ms": t_adj,
           "grad_over_forward": (t_fwd + t_adj) / t_fwd, "reverse_over_forward": t_adj / t_fwd,
           "finite": finite, "J_rel_error_vs_fp64": abs(float(J.item()) - J64) / abs(J64),
           "grad_rel_l2_error_vs_fp64": float(torch.linalg.norm(g - g64) / torch.linalg.norm(g64))}
    return out


def copy_probe(torch, P, nbytes=1 << 30, reps=20):
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
    return {"bytes_moved": 2 * nbytes, "us": ms * 1e3, "GBs": 2 * nbytes / (ms * 1e-3) / 1e9, "ok": ok}


def cpu_baseline(VX, EToV, c, N, q0, dt, sample_steps):
    from threadpoolctl import threadpool_info

    from oracle import dg
    prob = dg.Problem(VX, EToV, N, c)
    t0 = time.perf_counter()
    prob.lsrk4(q0, dt, sample_steps)
    sec = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    K, Np = prob.K, prob.Np
    return {
        "value": 4.0 * K * Np * 5 * sample_steps / sec,
        "unit": "DoF-stage/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "%d LSRK4 step(s) = %d stages of the FP64 dense-operator oracle on the full "
                  "K=%d, N=%d mesh (%.1f s)" % (sample_steps, 5 * sample_steps, K, N, sec),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", help="named workload (c1..c3)")
    ap.add_argument("--order", type=int, default=None, help="override N")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=1)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-nodal", action="store_true", help="skip the dense nodal comparator")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-shot batched workload")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--no-gradient", action="store_true", help="skip the misfit-gradient workload")
    ap.add_argument("--gradient-steps", type=int, default=500)
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--copy-probe-only", action="store_true",
                    help="only run the streaming-copy probe (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver runs on a single GPU; multi-GPU runs (--gpus %d) are not "
              "supported by this build" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1512_06025_amd as P
    import workload
    from paper_1512_06025_amd import ic

    if args.copy_probe_only:
        print(json.dumps({"copy_probe": copy_probe(torch, P)}), flush=True)
        return

    over = {} if args.order is None else {"N": args.order}
    cfg, VX, EToV, c = workload.build_preset(args.config, **over)
    N, K, Np, dt = cfg["N"], cfg["K"], cfg["Np"], cfg["dt"]
    Nfp = (N + 1) * (N + 2) // 2
    mesh = P.mesh_geometry(VX, EToV)
    q0 = ic.initial_state(N, VX, EToV, workload.INITIAL_FIELDS[cfg["ic"]])

    stages = 5 * args.steps
    dof = 4.0 * K * Np
    ms64, ok64, q64 = time_gpu(P, torch, N, mesh, c, q0, dt, args.steps, args.warmup, "f64")
    value = dof * stages / (ms64 * 1e-3)
    stage_us = ms64 * 1e3 / stages
    bytes_launch = algorithmic_bytes_per_element(N, 8) * K
    achieved = bytes_launch / (stage_us * 1e-6) / 1e9

    out = {
        "metric": "DoF-stage updates/s & % HBM roofline (BB vs nodal, FP64/FP32); grad/forward x",
        "value": value,
        "unit": "DoF-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "BB-DG acoustic forward, unit cube %d^3x6 = %d tets%s, N=%d (Np=%d), %s IC, "
                        "rigid walls, LSRK4 dt=%.6g, %d steps" % (
                            cfg["n"], K, ", interior vertices jittered +-%g h" % cfg["jitter"] if cfg["jitter"] else "",
                            N, Np, cfg["ic"], dt, args.steps),
            "K": K, "N": N, "Np": Np, "Nfp": Nfp, "stages": stages,
            "parallelism": "single GPU",
        },
        "stage_us": stage_us,
        "finite": ok64,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": recorded_traffic(stage_kernel_name(N, K), args.config),
            "kernel": stage_kernel_name(N, K),
            "bytes_per_launch": bytes_launch,
            "avg_launch_us": stage_us,
        },
    }
    if not args.no_fp32:
        ms32, ok32, q32 = time_gpu(P, torch, N, mesh, c, q0, dt, args.steps, args.warmup, "f32")
        st32 = ms32 * 1e3 / stages
        a32 = algorithmic_bytes_per_element(N, 4) * K / (st32 * 1e-6) / 1e9
        # both runs did warm-up + steps steps from q0; the FP64 path matches the oracle to 1e-12
        err32 = float(torch.linalg.norm(q32.double() - q64) / torch.linalg.norm(q64))
        out["fp32"] = {"value": dof * stages / (ms32 * 1e-3), "ms_per_step": ms32 / args.steps,
                       "stage_us": st32, "achieved_GBs": a32, "frac": a32 / HBM_PEAK_GBS, "finite": ok32,
                       "rel_l2_error_vs_fp64": err32}
    if not args.no_nodal:
        x0 = ic.initial_state(N, VX, EToV, workload.INITIAL_FIELDS[cfg["ic"]], basis="nodal")
        nod = {}
        for dt_name, bb_ms in (("f64", ms64), ("f32", out.get("fp32", {}).get("ms_per_step", 0) * args.steps)):
            if dt_name == "f32" and args.no_fp32:
                continue
            msn, okn, _ = time_gpu(P, torch, N, mesh, c, x0, dt, args.steps, args.warmup, dt_name, basis="nodal")
            flop = K * (24 * Np * Np + 32 * Np * Nfp)  # dense volume + lift per stage
            nod[dt_name] = {"value": dof * stages / (msn * 1e-3), "stage_us": msn * 1e3 / stages,
                            "tflops": flop * stages / (msn * 1e-3) / 1e12, "finite": okn,
                            "bb_speedup": msn / bb_ms}
        out["nodal"] = nod
    if not args.no_batched:
        out["batched"] = time_batched(P, torch, workload, args.batched_steps)
    if not args.no_gradient:
        out["gradient"] = time_gradient(P, torch, workload, args.gradient_steps)
    if not args.no_copy_probe:
        cp = copy_probe(torch, P)
        out["roofline"]["copy_probe_GBs"] = cp["GBs"]
        out["roofline"]["frac_of_copy_probe"] = achieved / cp["GBs"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(VX, EToV, c, N, q0, dt, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

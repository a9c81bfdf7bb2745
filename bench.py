#!/usr/bin/env python3
"""Benchmark of the SWR hot path on one MI355X.

Workload (the largest single-GPU shape): x in [0,1) periodic with
Nx = 4096, v in [-1,1] with Nv = 4096, T = 1, Nt = 8192, J = 32 equal
v-subdomains, overlap 2 cells, Robin transmission p = 8; f and u0 each a
sum of 16 Fourier x Legendre modes with N(0,1) coefficients from seed 0
(FP64).  One step = one SWR iteration: every subdomain marched over the
whole window (transport, source, implicit v-diffusion), the interface
traces exchanged and the residual (6.12) reduced.  K steps are one call
with K iterations, from zero initial traces, inputs resident in HBM.

Prints ONE JSON line.  `value` is subdomain cell-steps per second over the
timed iterations.  The roofline block is for the dominant kernel (the march
kernel), its average launch duration timed live with HIP events on the
stream its launches run on: `achieved` is the kernel's compulsory HBM bytes
per launch (state in and out, the source rows, the incoming traces of the
launch's levels, the interface-node values it writes) over that duration,
against the 8 TB/s HBM peak; `traffic` is what the HBM counters saw per
launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated by a copy kernel),
null when the kernel sources differ from those the counters were taken on.
Beside it: the FP64 rate of the same launches against the 78.6 TFLOP/s
vector peak, the VALU-busy share of the counter profile, and the copy
bandwidth the library's copy kernel reaches on this GPU.

Also reported once, beside the timed iterations: the time to an absolute
residual of 1e-10 in the parallel order from zero traces, from the u0
extension and from a learned guess (trained here on coarse solves of the
same J, overlap, T and p, carried to the full grid through the traces'
x-Fourier coefficients), and in red-black order on 32 time windows (each
from the extension of its start state); the HBM fraction of the same march
kernel taking one time step per launch (the fused step kernel in its
streaming form, `fused_one_step`), also against the copy kernel and against
a plain streaming kernel of the same tile shape (`kfp_tile_probe`); the
1024 x 1024, J = 8 solve to 1e-10 for p = 1, 2, 4, 8, 16 (`p_sweep_1024`); the
time to 1e-10 with and without learned initial traces on the learned-traces
shape (256 x 256, Nt = 512, J = 4), the network trained here on a bounded
number of seeded solves (`learned_guess`); and the oracle on the host cores
(a bounded sample of one iteration of the same shape, extrapolated).  `--scheme fem` times the paper's finite-element
discretisation instead.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NX = NV = 4096
NT, T = 8192, 1.0
J, OVERLAP, TR = 32, 2, 1
P_MAIN = 8.0
TOL = 1e-10
HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6
SIMDS, CLOCK_GHZ = 1024, 2.4  # 256 compute units x 4 SIMDs
# FP64 flops per cell-step: transport + source (1 mul, 2 fma), forward
# elimination (1 fma), back substitution (1 fma), segment correction (2 fma)
FLOPS_PER_CELL_STEP = 13.0
# time windows of the red-black solve to tolerance reported beside the
# timed iterations (4, 8, 16, 32 windows measured 9.0, 7.5, 6.8, 6.4 s at
# this shape)
N_WINDOWS = 32
# Counter profile of the march kernel at this workload (rocprofv3 --pmc,
# one pass per counter set; profiles/march_kernel_4096x4096_J32_Nt8192.md):
# HBM bytes per launch from FETCH_SIZE and WRITE_SIZE, each scaled by what
# the counter reads for the library's copy kernel of a known size, and the
# VALU instructions per launch.  Valid only for the kernel sources and
# launch configuration they were measured on; otherwise reported as null.
COUNTERS = {
    "config": (8, 17, 15, 1, 1),  # waves, seg_max, steps, groups, tiles
    "sha256": {
        "paper_1306_4596_amd/csrc/swr_kernels.hip":
            "6dbe1688911197c71c63445bfa425e057fccaca2dd0c94b16e34a61795571af5",
        "paper_1306_4596_amd/csrc/kfp_internal.h":
            "377909b348878a0016731dddcb594c302ce5fcad78a799486bec46768e69b477",
    },
    # mean over the 547 dispatches of one iteration: FETCH_SIZE 162705.71 KiB
    # (x 1048576 / 524302.22, its reading for 1 GiB copied), WRITE_SIZE
    # 224562.33 KiB (x 1048576 / 1048576.0)
    "read_bytes": 162705.706 * 1024 * (1048576.0 / 524302.219),
    "write_bytes": 224562.331 * 1024 * (1048576.0 / 1048576.0),
    "valu_insts": 66870632.75,  # SQ_INSTS_VALU per dispatch (wave instructions)
}


def counters_valid(config):
    if COUNTERS["config"] is None or tuple(config) != tuple(COUNTERS["config"]):
        return False
    for rel, digest in COUNTERS["sha256"].items():
        with open(os.path.join(ROOT, rel), "rb") as fp:
            if hashlib.sha256(fp.read()).hexdigest() != digest:
                return False
    return True


def compulsory_bytes_per_launch(rows, steps):
    """HBM bytes a launch of `steps` time steps cannot avoid: every unknown
    row's state read and written once and its source row read once, the two
    incoming trace planes of every interface at the launch's levels, and the
    six interface-node values per interface and level it writes (Robin)."""
    per_level = 2 * (J - 1) + 6 * (J - 1)
    return 8.0 * NX * (3.0 * rows + per_level * steps)


def optional(name, fn, *a):
    """Runs one reported-beside leg; a failure is recorded in its place
    (and on stderr) instead of ending the run before the JSON line."""
    try:
        return fn(*a)
    except Exception as e:  # noqa: BLE001 - any failure of a side leg
        progress(f"{name} failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def progress(msg):
    """A line on stderr as each part of the run finishes (stdout carries
    only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed SWR iterations")
    ap.add_argument("--warmup", type=int, default=2, help="untimed SWR iterations first")
    ap.add_argument("--no-solves", action="store_true", help="skip the time-to-tolerance solves")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess leg")
    ap.add_argument("--learned-train", type=int, default=1024,
                    help="training solves of the learned-guess leg")
    ap.add_argument("--learned-eval", type=int, default=64,
                    help="held-out seeds of the learned-guess leg")
    ap.add_argument("--no-learned-large", action="store_true",
                    help="skip the u0-extension and learned starts of the benchmark shape")
    ap.add_argument("--learned-large-train", type=int, default=256,
                    help="coarse training solves of the benchmark shape's learned guess")
    ap.add_argument("--scheme", choices=["fd", "fem"], default="fd")
    ap.add_argument("--copy-probe-mb", type=int, default=1024,
                    help="size of the copy-kernel bandwidth probe (MiB)")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fp:
            for line in fp:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(gpu_iters):
    """The oracle, as it stands, on the host cores: one SWR iteration of the
    same shape over the first steps of the window (same dt), on all threads
    and on one, extrapolated to a whole iteration and to the GPU's iteration
    count to 1e-10."""
    import oracle
    from paper_1306_4596_amd import inputs

    u0, f = inputs.random_fields(0, NX, NV)
    rows = (NV - 1) + (J - 1) * (OVERLAP + 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))

    def run(nthreads, nt_s):
        oracle.set_threads(nthreads)
        t0 = time.perf_counter()
        oracle.swr_solve(u0, f, T * nt_s / NT, nt_s, J, OVERLAP, TR, p=P_MAIN, tol=1e-300,
                         max_iter=1)
        dt = time.perf_counter() - t0
        return float(nt_s) * NX * rows / dt, dt

    rate, dt = run(threads, 96)
    rate1, dt1 = run(1, 12)
    oracle.set_threads(threads)
    per_iter = float(NT) * NX * rows / rate
    return {"value": rate, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"1 SWR iteration of 4096x4096 J=32 Robin p=8 over the first 96 of 8192 "
                      f"steps on {threads} threads ({96 * NX * rows:.3e} cell-steps, {dt:.1f} s); "
                      f"the same over 12 steps on 1 thread ({dt1:.1f} s)",
            "one_core": {"value": rate1, "unit": "cell-steps/s", "cores": 1},
            "cpu_model": cpu_model(), "compiler": "gcc -O3 -fopenmp",
            "extrapolated_iteration_s": per_iter,
            "extrapolated_time_to_tol_s": None if gpu_iters is None else per_iter * gpu_iters,
            "extrapolated_with_iterations": gpu_iters}


def large_starts(U0, F, zero, ntrain):
    """The benchmark shape solved to 1e-10 in the parallel order from the
    u0 extension and from the learned guess: linear BF16 stages trained
    inside this run on `ntrain` coarse solves (512 x 512 x 1024, the same
    J, overlap, T and p; seeds 1..ntrain, the workload's seed 0 held out),
    predicting the x-Fourier coefficients of the traces, evaluated on the
    full grid by kfp_trace_synth.  Times include the guess."""
    import torch

    import paper_1306_4596_amd as kfp
    from paper_1306_4596_amd import inputs, workloads

    out = {}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lam0 = kfp.u0_guess(U0, NT, J, OVERLAP, TR, P_MAIN)
    _, _, su = kfp.swr_solve(U0, F, T, NT, J, OVERLAP, TR, p=P_MAIN, tol=TOL, max_iter=1000,
                             lambda_init=lam0, history=False)
    torch.cuda.synchronize()
    out["parallel_u0"] = {"iters": su.iters, "seconds": round(time.perf_counter() - t1, 3),
                          "residual": su.residual}
    progress(f"parallel order from the u0 extension: {su.iters} iterations")
    del lam0
    kfp.release_workspace()
    g, rec = workloads.learned_large_guess(ntrain, log=progress)
    progress(f"coarse guess trained ({rec['generate_s']} s generating, {rec['train_s']} s training)")
    kfp.release_workspace()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lam0 = g.predict(inputs.coefficients(0), NT, NX)[0]
    _, _, sl = kfp.swr_solve(U0, F, T, NT, J, OVERLAP, TR, p=P_MAIN, tol=TOL, max_iter=1000,
                             lambda_init=lam0, history=False)
    torch.cuda.synchronize()
    secs = round(time.perf_counter() - t1, 3)
    out["parallel_learned"] = {"iters": sl.iters, "seconds": secs, "residual": sl.residual,
                               "training": rec}
    progress(f"parallel order from the learned guess: {sl.iters} iterations")
    out["time_saved_learned_vs_zero"] = 1.0 - secs / zero["seconds"]
    out["time_saved_learned_vs_u0"] = 1.0 - secs / out["parallel_u0"]["seconds"]
    del lam0, g
    kfp.release_workspace()
    torch.cuda.empty_cache()
    return out


def fused_one_step(U0, F, rows, copy_gbps):
    """The same shape with the multi-tile march kernel taking ONE time step
    per launch (8 wavefronts x 17 rows, one tile, a halo of one column): the
    fused step kernel in its streaming form, every cell-step moving its
    state and source through HBM.  One timed iteration (8192 launches);
    compulsory bytes per launch over the live average launch duration,
    against the 8 TB/s peak, the copy kernel's rate and the streaming rate
    of a plain kernel with the same tile shape (kfp_tile_probe)."""
    import torch

    import paper_1306_4596_amd as kfp

    kfp.set_config(8, 17, 1, 1, 1)
    try:
        kfp.swr_solve(U0, F, T, NT, J, OVERLAP, TR, p=P_MAIN, tol=1e-300, max_iter=1,
                      history=False)  # plan and graphs
        torch.cuda.synchronize()
        _, _, st = kfp.swr_solve(U0, F, T, NT, J, OVERLAP, TR, p=P_MAIN, tol=1e-300, max_iter=1,
                                 history=False)
        torch.cuda.synchronize()
    finally:
        kfp.set_config(0)
        kfp.release_workspace()
    launch_s = st.step_seconds / st.step_launches
    alg = compulsory_bytes_per_launch(rows, 1)
    gbps = alg / launch_s / 1e9
    progress(f"one step per launch: {launch_s * 1e6:.1f} us per launch, {gbps:.0f} GB/s")
    # the streaming ceiling of the same access shape: the library's tile probe
    # (state and source read, state written, no solve) over [nv+1][nx] arrays
    # in 8 wavefronts x 17 rows per 64-column tile, 20 launches on the
    # current stream
    V = torch.empty_like(U0)
    kfp.tile_probe(U0, F, V, 8, 17)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        nbytes = kfp.tile_probe(U0, F, V, 8, 17)
    e1.record()
    torch.cuda.synchronize()
    tile_gbps = nbytes / (e0.elapsed_time(e1) * 1e-3 / 20) / 1e9
    del V
    return {"kernel": "kfp::march_fd_kernel, 1 step per launch", "launches": st.step_launches,
            "avg_launch_us": round(launch_s * 1e6, 3), "alg_bytes_per_launch": alg,
            "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBPS, 4),
            "frac_of_copy": round(gbps / copy_gbps, 4) if copy_gbps else None,
            "tile_stream_GBps": round(tile_gbps, 1),
            "frac_of_tile_stream": round(gbps / tile_gbps, 4),
            "cell_steps_per_s": st.cell_steps / st.step_seconds}


def p_sweep():
    """The 1024 x 1024, Nt = 2000, T = 0.5, J = 8, overlap 2 shape (random
    fields seed 0) solved to 1e-10 from zero traces in the parallel order for
    each Robin parameter p in {1, 2, 4, 8, 16}: iterations and seconds."""
    import torch

    import paper_1306_4596_amd as kfp
    from paper_1306_4596_amd import inputs

    nx = nv = 1024
    u0, f = inputs.random_fields(0, nx, nv)
    U0, F = torch.from_numpy(u0).cuda(), torch.from_numpy(f).cuda()
    kfp.swr_solve(U0, F, 0.5, 2000, 8, 2, TR, p=8.0, tol=1e-300, max_iter=1)  # plan, graphs
    out = {"workload": "SWR 1024x1024 Nt=2000 T=0.5 J=8 overlap=2 Robin, seed 0, tol 1e-10"}
    for p in (1.0, 2.0, 4.0, 8.0, 16.0):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, st = kfp.swr_solve(U0, F, 0.5, 2000, 8, 2, TR, p=p, tol=TOL, max_iter=2000,
                                 history=False)
        torch.cuda.synchronize()
        out[f"p={p:g}"] = {"iters": st.iters, "seconds": round(time.perf_counter() - t1, 4),
                           "residual": st.residual}
    progress("p sweep at 1024 x 1024 done")
    kfp.release_workspace()
    return out


def learned_leg(ntrain, neval):
    """Time to 1e-10 with and without learned initial traces on the
    learned-traces shape (256 x 256, Nt = 512, T = 0.5, J = 4, overlap 2,
    Robin p = 4).  Two networks (BF16 weights, FP32 accumulation) are
    trained here, by the library's kernels, on `ntrain` solves the batch
    path generates: three linear stages (`linear`), and the same three
    linear stages followed by the 3 x 512 GELU network fitted to their
    remainder (`gelu`).  Every held-out seed is then solved from zero traces, from the
    u0 extension and from each network's traces (wall time of each call,
    inference included)."""
    import torch

    from paper_1306_4596_amd import learned

    shape = learned.SHAPE_256
    t0 = time.perf_counter()
    X, Y, _ = learned.generate(shape, range(ntrain), base="u0", log=progress)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    nets, t_train = {}, {}
    # a few thousand optimiser steps per linear stage (the map is linear and
    # well determined by ~1000 solves); the GELU network last, on what the
    # three linear stages leave, 10 epochs at a lower rate
    for name, kw, lrs, eps in (("linear", dict(depth=0, refine=2), [1e-3, 3e-3, 3e-3],
                                [200, 200, 200]),
                               ("gelu", dict(hidden=512, depth=3, skip=False, refine=2,
                                             gelu_last=True), [1e-3, 3e-3, 3e-3, 3e-4],
                                [200, 200, 200, 10])):
        g = learned.LearnedGuess(shape, **kw)
        t0 = time.perf_counter()
        g.fit(X, Y.clone() if name == "linear" else Y, batch=64, lrs=lrs, stage_epochs=eps)
        torch.cuda.synchronize()
        t_train[name] = round(time.perf_counter() - t0, 2)
        nets[name] = g
        progress(f"learned-traces shape: network {name} trained ({t_train[name]} s)")
    del X, Y
    ev = learned.evaluate(shape, range(20000, 20000 + neval), nets, log=progress)
    summ = learned.summarize(ev)
    keep = ("iters_mean", "iters_median", "seconds_mean", "seconds_median", "guess_err_median",
            "max_rel_l2_vs_zero_guess")
    out = {"workload": "SWR 256x256 Nt=512 T=0.5 J=4 overlap=2 Robin p=4, tol 1e-10",
           "networks": {"linear": "three BF16 linear stages",
                        "gelu": "three linear stages + 3x512 GELU stage on their remainder, BF16"},
           "train_seeds": ntrain, "eval_seeds": neval, "generate_s": round(t_gen, 2),
           "train_s": t_train}
    for k in ("zero", "u0", "linear", "gelu"):
        out[k] = {q: summ[k][q] for q in keep}
    for k in ("linear", "gelu"):
        out[f"time_saved_{k}_vs_zero"] = 1.0 - summ[k]["seconds_mean"] / summ["zero"]["seconds_mean"]
        out[f"time_saved_{k}_vs_u0"] = 1.0 - summ[k]["seconds_mean"] / summ["u0"]["seconds_mean"]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU "
                                   "decomposition is described in DESIGN.md and not run",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1306_4596_amd as kfp
    from paper_1306_4596_amd import inputs

    kfp.load_library()
    dev = torch.device("cuda:0")
    u0, f = inputs.random_fields(0, NX, NV)
    U0 = torch.from_numpy(u0).to(dev)
    F = torch.from_numpy(f).to(dev)
    del u0, f
    kfp.set_scheme(kfp.FEM if args.scheme == "fem" else kfp.FD)
    rows = kfp.subdomain_rows(NX, NV, NT, T, J, OVERLAP, TR)
    launch = kfp.get_launch_tiles(NX, NV, NT, T, J, OVERLAP, TR)  # waves, seg, steps, groups, tiles

    def iterate(k):
        return kfp.swr_solve(U0, F, T, NT, J, OVERLAP, TR, p=P_MAIN, tol=1e-300, max_iter=k,
                             history=False)

    # the copy kernel's bandwidth on this GPU (read + write of the buffer)
    copy_gbps = None
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        kfp.bw_probe(a, b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nbytes = kfp.bw_probe(a, b)
        e1.record()
        torch.cuda.synchronize()
        copy_gbps = 2.0 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del a, b
    if args.warmup > 0:
        iterate(args.warmup)
    torch.cuda.synchronize()
    progress(f"warm-up done ({args.warmup} iterations)")
    t0 = time.perf_counter()
    _, _, st = iterate(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"timed {args.steps} iterations: {wall:.3f} s")
    if st.iters != args.steps:
        raise SystemExit(f"expected {args.steps} iterations, ran {st.iters}")
    value = st.cell_steps / wall
    # the dominant kernel: its launches and their average duration come from
    # the library's HIP events around the time-step graph of each iteration,
    # on the stream the graphs run on
    launches = st.step_launches
    avg_launch_s = st.step_seconds / launches
    steps_per_launch = NT * st.iters / launches
    cells_launch = st.cell_steps / launches
    alg_bytes = compulsory_bytes_per_launch(rows, steps_per_launch)
    achieved = alg_bytes / avg_launch_s / 1e9
    if achieved > HBM_PEAK_GBPS:
        raise SystemExit(f"compulsory bytes above the HBM peak: {achieved:.0f} GB/s")
    fp64 = FLOPS_PER_CELL_STEP * cells_launch / avg_launch_s / 1e12
    have = counters_valid(launch) and args.scheme == "fd"
    tbytes = (COUNTERS["read_bytes"] + COUNTERS["write_bytes"]) if have else None
    valu_busy = (COUNTERS["valu_insts"] * 4.0 / (avg_launch_s * CLOCK_GHZ * 1e9 * SIMDS)
                 if have else None)
    kname = ("kfp::march_fd_kernel" if launch[4] > 0 else
             ("kfp::march_kernel" if launch[2] >= 1 else "kfp::step_kernel"))
    roof = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": round(tbytes / avg_launch_s / 1e9, 1) if tbytes else None,
            "traffic_bytes_per_launch": tbytes,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "launches": launches, "steps_per_launch": round(steps_per_launch, 3),
            "cell_steps_per_launch": cells_launch,
            "copy_kernel_GBps": round(copy_gbps, 1) if copy_gbps else None,
            "frac_of_copy": round(achieved / copy_gbps, 4) if copy_gbps else None,
            "fp64_tflops": round(fp64, 3), "fp64_frac": round(fp64 / FP64_PEAK_TFLOPS, 4),
            "flops_per_cell_step": FLOPS_PER_CELL_STEP,
            "valu_busy": round(valu_busy, 4) if valu_busy else None,
            "exchange_share_of_device_time": round(1.0 - st.step_seconds / st.device_seconds, 4)}
    out = {
        "metric": "subdomain cell-timesteps/sec",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "SWR Kolmogorov 4096x4096 Nt=8192 T=1 J=32 overlap=2 Robin p=8, "
                               "one SWR iteration per step, random Fourier-Legendre f,u0 seed 0",
                   "nx": NX, "nv": NV, "nt": NT, "T": T, "J": J, "overlap": OVERLAP,
                   "p": P_MAIN, "rows": rows,
                   "launch": {"waves": launch[0], "seg_max": launch[1], "steps": launch[2],
                              "groups": launch[3], "tiles": launch[4]},
                   "scheme": "finite differences" if args.scheme == "fd" else "finite elements"},
        "device_s_per_step": st.device_seconds / args.steps,
        "roofline": roof,
    }
    gpu_iters = None
    if not args.no_solves:
        solves = {}
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, s0 = kfp.swr_solve(U0, F, T, NT, J, OVERLAP, TR, p=P_MAIN, tol=TOL, max_iter=1000,
                                 history=False)
        torch.cuda.synchronize()
        gpu_iters = s0.iters
        solves["parallel_zero"] = {"iters": s0.iters, "seconds": round(time.perf_counter() - t1, 3),
                                   "residual": s0.residual}
        progress(f"parallel order from zero: {s0.iters} iterations")
        if not args.no_learned_large:
            r = optional("u0 and learned starts", large_starts, U0, F, solves["parallel_zero"],
                         args.learned_large_train)
            solves.update(r if "error" not in r else {"learned_starts": r})
        kfp.set_ordering(kfp.RED_BLACK)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, its, s1 = kfp.swr_solve_windows(U0, F, T, NT, J, OVERLAP, TR, p=P_MAIN, tol=TOL,
                                           max_iter=1000, n_windows=N_WINDOWS, guess=True)
        torch.cuda.synchronize()
        solves[f"red_black_{N_WINDOWS}_windows_u0"] = {"iters": its,
                                            "seconds": round(time.perf_counter() - t1, 3),
                                            "residual": s1.residual}
        progress(f"red-black order on {N_WINDOWS} windows: {sum(its)} iterations")
        kfp.set_ordering(kfp.PARALLEL)
        out["time_to_tol"] = {"tol": TOL, **solves}
    if not args.no_solves:
        out["fused_one_step"] = optional("one step per launch", fused_one_step, U0, F, rows,
                                         copy_gbps)
        out["p_sweep_1024"] = optional("p sweep", p_sweep)
    if not args.no_learned:
        del U0, F
        kfp.release_workspace()
        torch.cuda.empty_cache()
        out["learned_guess"] = optional("learned-traces leg", learned_leg, args.learned_train,
                                        args.learned_eval)
    if not args.no_cpu:
        out["cpu_baseline"] = optional("CPU baseline", cpu_baseline, gpu_iters)
        progress("CPU baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Throughput of the SWR path on the workloads beside the benchmark one.

    python -m paper_1306_4596_amd.workloads batch [--n 256] [--order 0|1] [--scheme fd|fem] [--tune]
    python -m paper_1306_4596_amd.workloads medium [--configs 8,17,16] [--scheme fd|fem]
    python -m paper_1306_4596_amd.workloads large [--iters 1] [--configs 8,17,16 8,17,8] [--scheme fd|fem]
    python -m paper_1306_4596_amd.workloads large-solve
    python -m paper_1306_4596_amd.workloads tile-probe

`batch`: uneven instances (Nx, Nv from {128, 256, 512, 1024}, J from
{2, 4, 8, 16}, Nt = 512, T = 0.25, overlap 2, Robin p = 4) solved together
by kfp_swr_batch to 1e-10, in the parallel order or (--order 1) red-black.
`medium`: Nx = Nv = 1024, Nt = 2000, T = 0.5, J = 8, overlap 2, Robin p = 8
solved to 1e-10 from zero traces.  `large`: Nx = Nv = 4096, Nt = 8192, T = 1, J = 32,
overlap 2, Robin p = 8, a fixed number of SWR iterations, once per launch
configuration.  `large-solve`: the same shape solved to 1e-10 from zero
traces and from the u0 extension, in the parallel and the red-black order,
and on 4 time windows.  `tile-probe`: the streaming rate of the tile
shapes of the register march (kfp_tile_probe) over [4188][4096] arrays,
beside the copy kernel.  `--scheme fem` runs `batch` or `large` with the
paper's finite-element discretisation instead of finite differences.  Each
prints one JSON line per measurement.  Inputs are seeded and synthetic
(inputs.py).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import binding as kb
from . import inputs


_SCHEME = [0]


def _scheme():
    return _SCHEME[0]


def run_batch(n: int, reps: int = 2, order: int = 0, tune: bool = False):
    import torch

    kb.set_ordering(order)
    specs = inputs.batch_specs(n)
    insts = []
    for sp in specs:
        u0, f = inputs.fields_from_coefficients(sp["coef"], sp["nx"], sp["nv"])
        insts.append(dict(u0=torch.from_numpy(u0).cuda(), f=torch.from_numpy(f).cuda(),
                          T=sp["T"], nt=sp["nt"], J=sp["J"], overlap=sp["overlap"], tr=kb.ROBIN,
                          p=sp["p"]))
    if tune:
        t0 = time.perf_counter()
        heights = kb.tune_batch(insts, iters=2)
        kb.reload_tune_cache()
        print(json.dumps({"tuned_heights": heights, "tune_s": time.perf_counter() - t0}),
              flush=True)
    for rep in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, rc = kb.swr_batch(insts, tol=1e-10, max_iter=400)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        cells = sum(r[2].cell_steps for r in res)
        its = [r[2].iters for r in res]
        classes = sorted(set(kb.get_batch_launch(d) for d in insts))
        print(json.dumps({"workload": f"batch of {n} uneven SWR instances", "order": order,
                          "tuned": tune, "classes": classes,
                          "scheme": "fem" if kb.FEM == _scheme() else "fd",
                          "rep": rep, "status": rc,
                          "wall_s": wall, "device_s": res[0][2].device_seconds,
                          "cell_steps": cells, "cell_steps_per_s": cells / wall,
                          "iters_min": min(its), "iters_mean": float(np.mean(its)),
                          "iters_max": max(its)}), flush=True)


def run_large(iters: int, configs):
    import torch

    nx = nv = 4096
    nt, T, J, o, p = 8192, 1.0, 32, 2, 8.0
    u0, f = inputs.random_fields(0, nx, nv)
    U0 = torch.from_numpy(u0).cuda()
    F = torch.from_numpy(f).cuda()
    del u0, f
    rows = kb.subdomain_rows(nx, nv, nt, T, J, o, kb.ROBIN)
    for cfg in configs:
        if cfg is not None:
            kb.set_config(*cfg)
        used = kb.get_launch_tiles(nx, nv, nt, T, J, o, kb.ROBIN)
        t0 = time.perf_counter()
        _, _, st = kb.swr_solve(U0, F, T, nt, J, o, kb.ROBIN, p=p, tol=1e-300, max_iter=iters)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print(json.dumps({"workload": "4096x4096 Nt=8192 T=1 J=32 overlap=2 Robin p=8",
                          "scheme": "fem" if kb.FEM == _scheme() else "fd",
                          "iterations": st.iters, "config": used, "rows": rows,
                          "wall_s_incl_setup": wall, "device_s": st.device_seconds,
                          "step_kernel_s": st.step_seconds,
                          "cell_steps_per_s": st.cell_steps / st.device_seconds,
                          "streaming_equivalent_GBps": 24.0 * st.cell_steps / st.step_seconds / 1e9}),
              flush=True)
        kb.release_workspace()
    kb.set_config(0)


def run_medium(configs, reps: int = 2):
    """The 1024 x 1024, Nt = 2000, T = 0.5, J = 8, overlap 2, Robin p = 8
    shape (seed 0) solved to 1e-10 from zero traces, once per launch
    configuration, after one untimed solve."""
    import torch

    nx = nv = 1024
    nt, T, J, o, p = 2000, 0.5, 8, 2, 8.0
    u0, f = inputs.random_fields(0, nx, nv)
    U0 = torch.from_numpy(u0).cuda()
    F = torch.from_numpy(f).cuda()
    rows = kb.subdomain_rows(nx, nv, nt, T, J, o, kb.ROBIN)
    # the library's copy kernel over 1 GiB: a known byte count for scaling
    # HBM counters taken on this run
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    kb.bw_probe(a, torch.empty_like(a))
    del a
    for cfg in configs:
        if cfg is not None:
            kb.set_config(*cfg)
        used = kb.get_launch_tiles(nx, nv, nt, T, J, o, kb.ROBIN)
        for rep in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st = kb.swr_solve(U0, F, T, nt, J, o, kb.ROBIN, p=p, tol=1e-10, max_iter=1000)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            print(json.dumps({"workload": "1024x1024 Nt=2000 T=0.5 J=8 overlap=2 Robin p=8 to 1e-10",
                              "scheme": "fem" if kb.FEM == _scheme() else "fd", "rep": rep,
                              "iterations": st.iters, "residual": st.residual, "config": used,
                              "rows": rows, "wall_s": wall, "device_s": st.device_seconds,
                              "step_kernel_s": st.step_seconds,
                              "step_launch_us": st.step_seconds / max(st.step_launches, 1) * 1e6,
                              "cell_steps_per_s": st.cell_steps / wall}),
                  flush=True)
        kb.release_workspace()
    kb.set_config(0)


def run_tile_probe(rows: int = 4188, nx: int = 4096, reps: int = 20):
    """Streaming rate of kfp_tile_probe (state and source read, state
    written) over [rows][nx] FP64 arrays in each built tile shape, against
    the library's copy kernel over 1 GiB."""
    import torch

    g = torch.Generator(device="cuda").manual_seed(0)
    U = torch.rand((rows, nx), generator=g, device="cuda", dtype=torch.float64)
    F = torch.rand((rows, nx), generator=g, device="cuda", dtype=torch.float64)
    V = torch.empty_like(U)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def rate(fn):
        fn()
        e0.record()
        for _ in range(reps):
            nbytes = fn()
        e1.record()
        torch.cuda.synchronize()
        return nbytes / (e0.elapsed_time(e1) * 1e-3 / reps) / 1e12

    out = {"workload": f"tile probe [{rows}][{nx}] FP64, {reps} launches each",
           "copy_1GiB_TBps": round(rate(lambda: 2 * kb.bw_probe(a, b)), 3)}
    for waves, rpw in ((8, 17), (8, 9), (4, 1)):
        out[f"{waves}x{rpw}_TBps"] = round(rate(lambda: kb.tile_probe(U, F, V, waves, rpw)), 3)
    print(json.dumps(out), flush=True)


def learned_large_guess(n_train, coarse=None, log=None):
    """The learned guess of the 4096 x 4096 workload: a modal guess trained
    on `n_train` coarse solves (seeds 1..n_train; the workload's own seed 0
    is held out).  Returns the guess and a JSON-ready record."""
    from . import learned

    c = coarse or learned.SHAPE_4096_COARSE
    g, t_gen, t_train, cit = learned.train_modal_guess(c, range(1, n_train + 1), log=log)
    rec = {"coarse_grid": [c.nx, c.nv, c.nt], "train_seeds": n_train, "generate_s": round(t_gen, 2),
           "train_s": round(t_train, 2), "coarse_iters_mean": cit,
           "network": "linear BF16 stages on the x-Fourier coefficients of the coarse traces",
           "modes": list(g.modes)}
    return g, rec


def run_large_solve(learned_train=0, orders=(0, 1), windows=(4,)):
    import torch

    nx = nv = 4096
    nt, T, J, o, p = 8192, 1.0, 32, 2, 8.0
    g = None
    if learned_train > 0:
        g, rec = learned_large_guess(learned_train, log=lambda m: print(m, flush=True))
        print(json.dumps({"learned_guess": rec}), flush=True)
    u0, f = inputs.random_fields(0, nx, nv)
    U0 = torch.from_numpy(u0).cuda()
    F = torch.from_numpy(f).cuda()
    del u0, f
    coef0 = inputs.coefficients(0)
    for order in orders:
        kb.set_ordering(order)
        starts = (("zero", "u0") + (("learned",) if g else ()) +
                  tuple(f"windows{w}" for w in windows) + (("windows4_learned",) if g else ()))
        for guess in starts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if guess == "windows4_learned":  # each window from its levels of the guess
                lam0 = g.predict(coef0, nt, nx)[0]
                _, its, st = kb.swr_solve_windows(U0, F, T, nt, J, o, kb.ROBIN, p=p, tol=1e-10,
                                                  max_iter=400, n_windows=4, lambda_init=lam0)
                iters = its
                del lam0
            elif guess.startswith("windows"):  # each window from its start state's extension
                _, its, st = kb.swr_solve_windows(U0, F, T, nt, J, o, kb.ROBIN, p=p, tol=1e-10,
                                                  max_iter=400, n_windows=int(guess[7:]),
                                                  guess=True)
                iters = its
            else:
                if guess == "learned":
                    lam0 = g.predict(coef0, nt, nx)[0]
                else:
                    lam0 = kb.u0_guess(U0, nt, J, o, kb.ROBIN, p) if guess == "u0" else None
                _, _, st = kb.swr_solve(U0, F, T, nt, J, o, kb.ROBIN, p=p, tol=1e-10,
                                        max_iter=400, lambda_init=lam0, history=False)
                iters = st.iters
                del lam0
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            print(json.dumps({"workload": "4096x4096 Nt=8192 T=1 J=32 overlap=2 Robin p=8 to 1e-10",
                              "order": "red-black" if order else "parallel", "start": guess,
                              "iterations": iters, "residual": st.residual,
                              "time_to_tol_s": round(wall, 3),
                              "cell_steps_per_s": st.cell_steps / wall}), flush=True)
            kb.release_workspace()
    kb.set_ordering(0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["batch", "medium", "large", "large-solve", "tile-probe"])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--iters", type=int, default=1)
    ap.add_argument("--order", type=int, default=0, choices=[0, 1])
    ap.add_argument("--scheme", choices=["fd", "fem"], default="fd")
    ap.add_argument("--tune", action="store_true",
                    help="batch: tune its launch classes first (kfp_tune_batch; the cache is "
                         "$KFP_TUNE_CACHE)")
    ap.add_argument("--learned-train", type=int, default=0,
                    help="large-solve: also solve from a learned guess trained on this many "
                         "coarse solves")
    ap.add_argument("--orders", default="0,1", help="large-solve: solve orders (0 parallel, 1 red-black)")
    ap.add_argument("--windows", default="4",
                    help="large-solve: time-window counts of the windowed solves (comma-separated)")
    ap.add_argument("--configs", nargs="*", default=[],
                    help="launch configurations waves,seg,steps[,groups[,tiles]] (default: "
                         "the library's choice)")
    a = ap.parse_args()
    kb.load_library()
    _SCHEME[0] = kb.FEM if a.scheme == "fem" else kb.FD
    kb.set_scheme(_SCHEME[0])
    if a.which == "batch":
        run_batch(a.n, order=a.order, tune=a.tune)
    elif a.which == "tile-probe":
        run_tile_probe()
    elif a.which == "medium":
        run_medium([tuple(int(x) for x in c.split(",")) for c in a.configs] or [None])
    elif a.which == "large-solve":
        run_large_solve(a.learned_train, tuple(int(x) for x in a.orders.split(",") if x),
                        tuple(int(x) for x in a.windows.split(",") if x))
    else:
        cfgs = [tuple(int(x) for x in c.split(",")) for c in a.configs] or [None]
        run_large(a.iters, cfgs)


if __name__ == "__main__":
    main()

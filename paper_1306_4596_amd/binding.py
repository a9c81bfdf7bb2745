"""ctypes binding of libkfpswr (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(PKG, "_lib", "libkfpswr.so")

DIRICHLET = 0
ROBIN = 1

KFP_OK, KFP_EINVAL, KFP_ENOMEM, KFP_EDEVICE, KFP_ENOCONV = range(5)
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOCONV"}


class KfpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"kfp {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nv", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("T", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarted", ctypes.c_int32),
                ("residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("device_seconds", ctypes.c_double), ("step_seconds", ctypes.c_double),
                ("step_launches", ctypes.c_double),
                ("cell_steps", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("res_history", ctypes.POINTER(ctypes.c_double))]


class Instance(ctypes.Structure):
    _fields_ = [("g", Grid), ("J", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("tr", ctypes.c_int32), ("p", ctypes.c_double),
                ("u0", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("s", ctypes.POINTER(ctypes.c_double)), ("lambda_init", ctypes.c_void_p),
                ("uT", ctypes.c_void_p), ("lambda_out", ctypes.c_void_p),
                ("q", ctypes.c_double)]


class SWRStats:
    """Per-solve statistics returned by swr_solve / swr_batch."""

    def __init__(self, st: Stats, history):
        self.iters = st.iters
        self.restarted = bool(st.restarted)
        self.residual = st.residual
        self.seconds = st.seconds
        self.device_seconds = st.device_seconds
        self.step_seconds = st.step_seconds
        self.step_launches = st.step_launches
        self.cell_steps = st.cell_steps
        self.alg_bytes = st.alg_bytes
        self.res_history = history

    def __repr__(self):
        return (f"SWRStats(iters={self.iters}, residual={self.residual:.3e}, "
                f"seconds={self.seconds:.4f}, device_seconds={self.device_seconds:.4f})")


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Loads the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"libkfpswr is not built ({_LIB_PATH} missing); run "
            "`python -m paper_1306_4596_amd.build` (needs hipcc for gfx950)")
    # torch first: its HIP runtime then also serves the library (same soname);
    # loading the library first would bring a second runtime into the process
    import torch  # noqa: F401

    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    G = ctypes.POINTER(Grid)
    D = ctypes.POINTER(ctypes.c_double)
    lib.kfp_mono_solve.argtypes = [G, vp, vp, D, vp, vp]
    lib.kfp_mono_solve_static.argtypes = [G, vp, vp, D, vp, vp]
    lib.kfp_swr_solve.argtypes = [G, vp, vp, D, i32, i32, i32, f64, f64, i32, vp, vp, vp,
                                  ctypes.POINTER(Stats), vp]
    lib.kfp_swr_solve_pq.argtypes = [G, vp, vp, D, i32, i32, i32, f64, f64, f64, i32, vp, vp, vp,
                                     ctypes.POINTER(Stats), vp]
    lib.kfp_u0_guess_pq.argtypes = [G, vp, i32, i32, i32, f64, f64, vp, vp]
    lib.kfp_swr_solve_windows.argtypes = [G, vp, vp, D, i32, i32, i32, f64, f64, f64, i32, i32,
                                          i32, vp, ctypes.POINTER(i32), ctypes.POINTER(Stats),
                                          vp]
    lib.kfp_swr_solve_windows_init.argtypes = [G, vp, vp, D, i32, i32, i32, f64, f64, f64, i32,
                                               i32, vp, vp, ctypes.POINTER(i32),
                                               ctypes.POINTER(Stats), vp]
    lib.kfp_u0_guess.argtypes = [G, vp, i32, i32, i32, f64, vp, vp]
    lib.kfp_swr_batch.argtypes = [i32, ctypes.POINTER(Instance), f64, i32,
                                  ctypes.POINTER(Stats), vp]
    pi = ctypes.POINTER(i32)
    lib.kfp_tune.argtypes = [G, i32, i32, i32, f64, pi, pi, pi, vp]
    lib.kfp_set_config.argtypes = [i32, i32, i32]
    lib.kfp_set_launch.argtypes = [i32, i32, i32, i32]
    lib.kfp_set_launch_tiles.argtypes = [i32, i32, i32, i32, i32]
    lib.kfp_tune_batch.argtypes = [i32, ctypes.POINTER(Instance), i32, pi, vp]
    lib.kfp_get_batch_launch.argtypes = [ctypes.POINTER(Instance), pi, pi, pi, pi, pi]
    lib.kfp_get_launch_tiles.argtypes = [G, i32, i32, i32, pi, pi, pi, pi, pi]
    lib.kfp_get_launch.argtypes = [G, i32, i32, i32, pi, pi, pi, pi]
    lib.kfp_set_pipeline.argtypes = [i32]
    lib.kfp_set_ordering.argtypes = [i32]
    lib.kfp_set_scheme.argtypes = [i32]
    lib.kfp_set_kernel_timing.argtypes = [i32]
    lib.kfp_get_config.argtypes = [G, i32, i32, i32, pi, pi, pi]
    lib.kfp_subdomain_rows.argtypes = [G, i32, i32, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.kfp_bw_probe.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.kfp_tile_probe.argtypes = [vp, vp, vp, ctypes.c_int64, i32, i32, i32, vp]
    lib.kfp_last_error.restype = ctypes.c_char_p
    lib.kfp_last_error.argtypes = []
    lib.kfp_release_workspace.restype = None
    for name in ("kfp_mono_solve", "kfp_mono_solve_static", "kfp_swr_solve", "kfp_swr_solve_pq", "kfp_swr_solve_windows",
                 "kfp_swr_solve_windows_init",
                 "kfp_u0_guess",
                 "kfp_u0_guess_pq", "kfp_swr_batch", "kfp_tune",
                 "kfp_set_config", "kfp_set_launch", "kfp_get_launch", "kfp_set_pipeline",
                 "kfp_set_launch_tiles", "kfp_get_launch_tiles", "kfp_tune_batch",
                 "kfp_get_batch_launch",
                 "kfp_set_ordering", "kfp_set_scheme", "kfp_set_kernel_timing", "kfp_get_config", "kfp_subdomain_rows", "kfp_bw_probe",
                 "kfp_tile_probe"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st, allow_noconv=False):
    if st == KFP_OK or (allow_noconv and st == KFP_ENOCONV):
        return st
    msg = load_library().kfp_last_error().decode(errors="replace")
    raise KfpError(st, msg)


def _grid(nx, nv, nt, T):
    return Grid(int(nx), int(nv), int(nt), float(T))


def _ptr(t):
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError("tensors must live on the GPU")
    if t.dtype != torch.float64:
        raise ValueError("tensors must be float64")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host_s(s, nt):
    if s is None:
        return None, None
    import numpy as np

    arr = np.ascontiguousarray(np.asarray(s, dtype=np.float64))
    if arr.shape != (nt + 1,):
        raise ValueError(f"s must have nt+1 = {nt + 1} entries")
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _shape(u0):
    if u0.dim() != 2:
        raise ValueError("fields are [nv+1][nx]")
    return u0.shape[0] - 1, u0.shape[1]


def _expect(t, shape, name):
    """Raises ValueError unless tensor `t` (if given) has exactly `shape`: a
    mis-sized buffer would otherwise be read or written out of bounds by the
    kernels, which only see its pointer."""
    if t is None:
        return
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _check_fields(u0, f, nt, J, lambda_init=None, out=None):
    """Shapes of one SWR instance's inputs: f and out like u0 ([nv+1][nx]),
    lambda_init [2(J-1)][nt][nx].  Returns (nv, nx)."""
    nv, nx = _shape(u0)
    _expect(f, u0.shape, "f")
    _expect(out, u0.shape, "out")
    if lambda_init is not None:
        if int(J) < 2:
            raise ValueError("lambda_init is given but J < 2 has no interfaces")
        _expect(lambda_init, (2 * (int(J) - 1), int(nt), nx), "lambda_init")
    return nv, nx


def check_mlp_io(n_in, n_out, X, T=None, out=None):
    """Shapes of a network call: X [B][n_in], T and out [B][n_out].  Returns B."""
    if X.dim() != 2:
        raise ValueError(f"X must be [B][{n_in}], got shape {tuple(X.shape)}")
    B = int(X.shape[0])
    if B < 1:
        raise ValueError("the batch is empty")
    _expect(X, (B, n_in), "X")
    _expect(T, (B, n_out), "T")
    _expect(out, (B, n_out), "out")
    return B


def mono_solve(u0, f, T, nt, s=None, out=None, stream=None):
    """Monodomain discrete solution at t = T ([nv+1][nx] float64 on the GPU)."""
    import torch

    nv, nx = _check_fields(u0, f, nt, 1, out=out)
    uT = out if out is not None else torch.empty_like(u0)
    keep, sp = _host_s(s, nt)
    g = _grid(nx, nv, nt, T)
    _check(load_library().kfp_mono_solve(ctypes.byref(g), _ptr(u0), _ptr(f), sp, _ptr(uT),
                                         _stream(stream)))
    return uT


def mono_solve_static(u0, f, T, nt, s=None, out=None, stream=None):
    """mono_solve through the entry point that allocates nothing (its state
    and tables live in the library's static per-GPU workspace)."""
    import torch

    nv, nx = _check_fields(u0, f, nt, 1, out=out)
    uT = out if out is not None else torch.empty_like(u0)
    keep, sp = _host_s(s, nt)
    g = _grid(nx, nv, nt, T)
    _check(load_library().kfp_mono_solve_static(ctypes.byref(g), _ptr(u0), _ptr(f), sp,
                                                _ptr(uT), _stream(stream)))
    return uT


def swr_solve(u0, f, T, nt, J, overlap, transmission, p=0.0, tol=1e-10, max_iter=200,
              lambda_init=None, s=None, want_lambda=False, history=True, stream=None,
              raise_noconv=False, q=None):
    """Parallel SWR solve.  Returns (uT, lambda or None, SWRStats).  q: the
    second Robin parameter of OSWR(p,q) (None: q = p)."""
    import numpy as np
    import torch

    nv, nx = _check_fields(u0, f, nt, J, lambda_init)
    uT = torch.empty_like(u0)
    lam = None
    if want_lambda and J > 1:
        lam = torch.empty((2 * (J - 1), nt, nx), dtype=torch.float64, device=u0.device)
    keep, sp = _host_s(s, nt)
    hist = np.zeros(max_iter) if history else None
    st = Stats()
    if hist is not None:
        st.res_history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    g = _grid(nx, nv, nt, T)
    lib = load_library()
    if q is None:
        rc = lib.kfp_swr_solve(ctypes.byref(g), _ptr(u0), _ptr(f), sp, int(J), int(overlap),
                               int(transmission), float(p), float(tol), int(max_iter),
                               _ptr(lambda_init), _ptr(uT), _ptr(lam), ctypes.byref(st),
                               _stream(stream))
    else:
        rc = lib.kfp_swr_solve_pq(ctypes.byref(g), _ptr(u0), _ptr(f), sp, int(J), int(overlap),
                                  int(transmission), float(p), float(q), float(tol),
                                  int(max_iter), _ptr(lambda_init), _ptr(uT), _ptr(lam),
                                  ctypes.byref(st), _stream(stream))
    _check(rc, allow_noconv=not raise_noconv)
    h = hist[: st.iters].copy() if hist is not None else None
    return uT, lam, SWRStats(st, h)


def swr_solve_windows(u0, f, T, nt, J, overlap, transmission, p=0.0, tol=1e-10, max_iter=200,
                      n_windows=1, s=None, q=None, guess=False, stream=None, lambda_init=None):
    """SWR on n_windows consecutive time windows (each from the glued end
    state of the one before).  lambda_init: traces of the whole [0, T]
    ([2(J-1)][nt][nx]); each window starts from its levels of them (guess is
    then ignored).  Returns (uT, per-window iteration counts, SWRStats summed
    over the windows)."""
    import numpy as np
    import torch

    nv, nx = _check_fields(u0, f, nt, J, lambda_init=lambda_init)
    if int(n_windows) < 1:
        raise ValueError("n_windows must be >= 1")
    uT = torch.empty_like(u0)
    keep, sp = _host_s(s, nt)
    its = (ctypes.c_int32 * int(n_windows))()
    st = Stats()
    g = _grid(nx, nv, nt, T)
    if lambda_init is not None:
        rc = load_library().kfp_swr_solve_windows_init(
            ctypes.byref(g), _ptr(u0), _ptr(f), sp, int(J), int(overlap), int(transmission),
            float(p), float(p if q is None else q), float(tol), int(max_iter), int(n_windows),
            _ptr(lambda_init), _ptr(uT), its, ctypes.byref(st), _stream(stream))
    else:
        rc = load_library().kfp_swr_solve_windows(
            ctypes.byref(g), _ptr(u0), _ptr(f), sp, int(J), int(overlap), int(transmission),
            float(p), float(p if q is None else q), float(tol), int(max_iter), int(n_windows),
            1 if guess else 0, _ptr(uT), its, ctypes.byref(st), _stream(stream))
    _check(rc, allow_noconv=True)
    return uT, [int(x) for x in its], SWRStats(st, None)


def u0_guess(u0, nt, J, overlap, transmission, p=0.0, stream=None, q=None):
    """Initial traces Q(u0) at every interface node and time level."""
    import torch

    nv, nx = _shape(u0)
    lam = torch.empty((2 * (J - 1), nt, nx), dtype=torch.float64, device=u0.device)
    g = _grid(nx, nv, nt, 0.5 * nt / nx)  # the traces do not depend on T; any CFL-valid T
    lib = load_library()
    if q is None:
        _check(lib.kfp_u0_guess(ctypes.byref(g), _ptr(u0), int(J), int(overlap),
                                int(transmission), float(p), _ptr(lam), _stream(stream)))
    else:
        _check(lib.kfp_u0_guess_pq(ctypes.byref(g), _ptr(u0), int(J), int(overlap),
                                   int(transmission), float(p), float(q), _ptr(lam),
                                   _stream(stream)))
    return lam


def swr_batch(instances, tol=1e-10, max_iter=200, history=False, stream=None):
    """Batched SWR.  `instances` is a list of dicts with keys u0, f, T, nt, J,
    overlap, tr, p and optionally q, s, lambda_init, want_lambda.  Returns a list
    of (uT, lambda or None, SWRStats) and the overall status (0 or 4)."""
    import numpy as np
    import torch

    n = len(instances)
    arr = (Instance * n)()
    keep = []
    outs = []
    stats = (Stats * n)()
    hists = []
    for i, d in enumerate(instances):
        u0, f = d["u0"], d["f"]
        nt, J = int(d["nt"]), int(d["J"])
        nv, nx = _check_fields(u0, f, nt, J, d.get("lambda_init"))
        uT = torch.empty_like(u0)
        lam = None
        if d.get("want_lambda") and J > 1:
            lam = torch.empty((2 * (J - 1), nt, nx), dtype=torch.float64, device=u0.device)
        sarr, sp = _host_s(d.get("s"), nt)
        keep.append(sarr)
        arr[i].g = _grid(nx, nv, nt, d["T"])
        arr[i].J = J
        arr[i].overlap = int(d["overlap"])
        arr[i].tr = int(d["tr"])
        arr[i].p = float(d.get("p", 0.0))
        arr[i].q = float(d["q"]) if d.get("q") is not None else 0.0
        arr[i].u0 = _ptr(u0).value
        arr[i].f = _ptr(f).value
        arr[i].s = sp
        li = d.get("lambda_init")
        arr[i].lambda_init = _ptr(li).value if li is not None else None
        arr[i].uT = _ptr(uT).value
        arr[i].lambda_out = _ptr(lam).value if lam is not None else None
        h = np.zeros(max_iter) if history else None
        if h is not None:
            stats[i].res_history = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        hists.append(h)
        outs.append((uT, lam))
    rc = load_library().kfp_swr_batch(n, arr, float(tol), int(max_iter), stats, _stream(stream))
    _check(rc, allow_noconv=True)
    res = []
    for i in range(n):
        h = hists[i][: stats[i].iters].copy() if hists[i] is not None else None
        res.append((outs[i][0], outs[i][1], SWRStats(stats[i], h)))
    return res, rc


def _instance_array(instances):
    """The C instance array of swr_batch-style dicts (outputs allocated):
    (array, buffers to keep alive, per-instance (uT, lambda or None))."""
    import torch

    n = len(instances)
    arr = (Instance * n)()
    keep, outs = [], []
    for i, d in enumerate(instances):
        u0, f = d["u0"], d["f"]
        nt, J = int(d["nt"]), int(d["J"])
        nv, nx = _check_fields(u0, f, nt, J, d.get("lambda_init"))
        uT = torch.empty_like(u0)
        lam = None
        if d.get("want_lambda") and J > 1:
            lam = torch.empty((2 * (J - 1), nt, nx), dtype=torch.float64, device=u0.device)
        sarr, sp = _host_s(d.get("s"), nt)
        keep.append(sarr)
        arr[i].g = _grid(nx, nv, nt, d["T"])
        arr[i].J = J
        arr[i].overlap = int(d["overlap"])
        arr[i].tr = int(d["tr"])
        arr[i].p = float(d.get("p", 0.0))
        arr[i].q = float(d["q"]) if d.get("q") is not None else 0.0
        arr[i].u0 = _ptr(u0).value
        arr[i].f = _ptr(f).value
        arr[i].s = sp
        li = d.get("lambda_init")
        arr[i].lambda_init = _ptr(li).value if li is not None else None
        arr[i].uT = _ptr(uT).value
        arr[i].lambda_out = _ptr(lam).value if lam is not None else None
        outs.append((uT, lam))
    return arr, keep, outs


def tune_batch(instances, iters=2, stream=None):
    """Tunes the launch classes of swr_batch for these instances (one class
    per subdomain height); caches the winners.  Returns the number of
    heights tuned."""
    arr, keep, outs = _instance_array(instances)
    k = ctypes.c_int32()
    _check(load_library().kfp_tune_batch(len(instances), arr, int(iters), ctypes.byref(k),
                                         _stream(stream)))
    return k.value


def get_batch_launch(instance):
    """(waves, seg_max, steps, groups, tiles) of the launch class swr_batch
    would run this instance (a swr_batch-style dict) in."""
    arr, keep, outs = _instance_array([instance])
    v = [ctypes.c_int32() for _ in range(5)]
    _check(load_library().kfp_get_batch_launch(arr, *[ctypes.byref(x) for x in v]))
    w, g_, s, k, tl = (x.value for x in v)
    return w, s, k, g_, tl


def tune(nx, nv, nt, T, J, overlap, transmission, p=1.0, stream=None):
    """Times the compiled launch configurations for one shape; caches the
    winner.  Returns (waves, seg_max, steps)."""
    w, s, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    g = _grid(nx, nv, nt, T)
    _check(load_library().kfp_tune(ctypes.byref(g), int(J), int(overlap), int(transmission),
                                   float(p), ctypes.byref(w), ctypes.byref(s), ctypes.byref(k),
                                   _stream(stream)))
    return w.value, s.value, k.value


def reload_tune_cache():
    """Forgets the tuning choices in memory; the next solve re-reads the
    cache file named by $KFP_TUNE_CACHE."""
    lib = load_library()
    lib.kfp_reload_tune_cache.restype = ctypes.c_int
    _check(lib.kfp_reload_tune_cache())


def set_config(waves=0, seg_max=0, steps=1, groups=1, tiles=0):
    """Forces a launch configuration (waves=0: automatic); groups > 1 splits
    each wavefront of the march kernel into lane groups; tiles 1 or 2 selects
    the multi-tile finite-difference march kernel."""
    _check(load_library().kfp_set_launch_tiles(int(waves), int(groups), int(seg_max), int(steps),
                                               int(tiles)))


def get_config(nx, nv, nt, T, J, overlap, transmission):
    """(waves, seg_max, steps) a solve of this shape would use."""
    w, s, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    g = _grid(nx, nv, nt, T)
    _check(load_library().kfp_get_config(ctypes.byref(g), int(J), int(overlap), int(transmission),
                                         ctypes.byref(w), ctypes.byref(s), ctypes.byref(k)))
    return w.value, s.value, k.value


def get_launch(nx, nv, nt, T, J, overlap, transmission):
    """(waves, seg_max, steps, groups) a solve of this shape would use."""
    w, g_, s, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    g = _grid(nx, nv, nt, T)
    _check(load_library().kfp_get_launch(ctypes.byref(g), int(J), int(overlap), int(transmission),
                                         ctypes.byref(w), ctypes.byref(g_), ctypes.byref(s),
                                         ctypes.byref(k)))
    return w.value, s.value, k.value, g_.value


def get_launch_tiles(nx, nv, nt, T, J, overlap, transmission):
    """(waves, seg_max, steps, groups, tiles) a solve of this shape would use."""
    v = [ctypes.c_int32() for _ in range(5)]
    g = _grid(nx, nv, nt, T)
    _check(load_library().kfp_get_launch_tiles(ctypes.byref(g), int(J), int(overlap),
                                               int(transmission), *[ctypes.byref(x) for x in v]))
    w, g_, s, k, tl = (x.value for x in v)
    return w, s, k, g_, tl


def subdomain_rows(nx, nv, nt, T, J, overlap, transmission):
    r = ctypes.c_int64()
    g = _grid(nx, nv, nt, T)
    _check(load_library().kfp_subdomain_rows(ctypes.byref(g), int(J), int(overlap),
                                             int(transmission), ctypes.byref(r)))
    return r.value


def bw_probe(src, dst, stream=None):
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
    nbytes -= nbytes % 16
    _check(load_library().kfp_bw_probe(ctypes.c_void_p(src.data_ptr()),
                                       ctypes.c_void_p(dst.data_ptr()), int(nbytes),
                                       _stream(stream)))
    return nbytes


def tile_probe(U, F, V, waves=8, rows_per_wave=17, stream=None):
    """V = U + F/2 over [rows][nx] FP64 tensors in the tile shape of the
    register march at one step per launch (kfp_tile_probe).  Returns the
    bytes moved (three streams of 8 B per cell)."""
    import torch

    for name, t in (("U", U), ("F", F), ("V", V)):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
            raise ValueError(f"{name} must be a contiguous 2-D float64 CUDA tensor")
    if tuple(F.shape) != tuple(U.shape) or tuple(V.shape) != tuple(U.shape):
        raise ValueError("U, F and V must have the same shape")
    rows, nx = int(U.shape[0]), int(U.shape[1])
    _check(load_library().kfp_tile_probe(_ptr(U), _ptr(F), _ptr(V), rows, nx, int(waves),
                                         int(rows_per_wave), _stream(stream)))
    return 24 * rows * nx


def set_pipeline(inflight=-1):
    """Overlapped SWR iterations: -1 automatic (default), 0 off, >= 2 in flight."""
    _check(load_library().kfp_set_pipeline(int(inflight)))


PARALLEL, RED_BLACK = 0, 1
FD, FEM = 0, 1


def set_ordering(order=PARALLEL):
    """Order of the subdomain solves in an iteration: PARALLEL (default) or
    RED_BLACK (even subdomains, then odd ones with the traces just sent)."""
    _check(load_library().kfp_set_ordering(int(order)))


def set_scheme(scheme=FD):
    """Discretisation of every later solve: FD (default; finite differences,
    IMEX step, zero values at v = +-1) or FEM (Section 6.2 as printed: linear
    finite elements with the consistent mass matrix, Neumann ends, the
    diffusion stage before the transport)."""
    _check(load_library().kfp_set_scheme(int(scheme)))


def set_kernel_timing(on=True):
    """HIP events around every time-step kernel launch of overlapped solves."""
    _check(load_library().kfp_set_kernel_timing(1 if on else 0))


def release_workspace():
    load_library().kfp_release_workspace()


# ------------------------------------------------------------- learned part --
def _fptr(t, dtype=None):
    import torch

    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _mlp_sigs(lib):
    if getattr(lib, "_mlp_sigs", False):
        return lib
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    pd = ctypes.POINTER(ctypes.c_double)
    lib.kfp_mlp_create.argtypes = [i32, i32, i32, i64, ctypes.c_uint64, ctypes.POINTER(vp)]
    lib.kfp_mlp_create_ex.argtypes = [i32, i32, i32, i64, i32, ctypes.c_uint64,
                                      ctypes.POINTER(vp)]
    lib.kfp_mlp_destroy.argtypes = [vp]
    lib.kfp_mlp_destroy.restype = None
    lib.kfp_mlp_forward.argtypes = [vp, i32, vp, vp, vp]
    lib.kfp_mlp_backward.argtypes = [vp, i32, vp, vp, pd, vp]
    lib.kfp_mlp_adam.argtypes = [vp, f32, vp]
    lib.kfp_mlp_train_step.argtypes = [vp, i32, vp, vp, f32, pd, vp]
    lib.kfp_mlp_layer_shape.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.kfp_mlp_param.argtypes = [vp, i32, i32, i32, vp, vp]
    lib.kfp_mlp_save.argtypes = [vp, ctypes.c_char_p]
    lib.kfp_mlp_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    lib.kfp_cast_f64_f32.argtypes = [vp, vp, vp, i64, vp]
    lib.kfp_column_stats.argtypes = [vp, i32, i64, f32, vp, vp, vp]
    lib.kfp_axpy_f32.argtypes = [vp, vp, f32, i64, vp]
    lib.kfp_mul_f32.argtypes = [vp, vp, i64, vp]
    lib.kfp_standardize.argtypes = [vp, i32, i64, vp, vp, vp]
    lib.kfp_destandardize.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp]
    pi32 = ctypes.POINTER(i32)
    lib.kfp_trace_modes.argtypes = [vp, i64, i32, i32, pi32, vp, vp]
    lib.kfp_trace_synth.argtypes = [vp, i32, i32, i32, pi32, i32, i32, vp, vp]
    lib.kfp_trace_modes.restype = ctypes.c_int
    lib.kfp_trace_synth.restype = ctypes.c_int
    for n in ("kfp_mlp_create", "kfp_mlp_create_ex", "kfp_mlp_forward", "kfp_mlp_backward", "kfp_mlp_adam",
              "kfp_mlp_train_step", "kfp_mlp_layer_shape", "kfp_mlp_param", "kfp_mlp_save",
              "kfp_mlp_load", "kfp_cast_f64_f32", "kfp_column_stats", "kfp_standardize",
              "kfp_destandardize", "kfp_axpy_f32", "kfp_mul_f32"):
        getattr(lib, n).restype = ctypes.c_int
    lib._mlp_sigs = True
    return lib


MLP_SKIP = 1


class MLP:
    """Handle of the library's network (BF16 weights, FP32 accumulation).
    skip=True: the output layer also reads the network input (a GELU trunk
    plus a linear map of the input)."""

    def __init__(self, n_in=64, hidden=512, depth=3, n_out=786432, seed=0, skip=False,
                 _handle=None):
        lib = _mlp_sigs(load_library())
        self._lib = lib
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib.kfp_mlp_create_ex(int(n_in), int(hidden), int(depth), int(n_out),
                                         MLP_SKIP if skip else 0, int(seed), ctypes.byref(h)))
            _handle = h
        self._h = _handle
        self.depth = self.layers() - 1

    @classmethod
    def load(cls, path):
        lib = _mlp_sigs(load_library())
        h = ctypes.c_void_p()
        _check(lib.kfp_mlp_load(str(path).encode(), ctypes.byref(h)))
        return cls(_handle=h)

    def save(self, path):
        _check(self._lib.kfp_mlp_save(self._h, str(path).encode()))

    def close(self):
        if self._h is not None and self._h.value:
            self._lib.kfp_mlp_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layers(self):
        n = 0
        i, o = ctypes.c_int32(), ctypes.c_int64()
        while self._lib.kfp_mlp_layer_shape(self._h, n, ctypes.byref(i), ctypes.byref(o)) == 0:
            n += 1
        return n

    def shape(self, layer):
        i, o = ctypes.c_int32(), ctypes.c_int64()
        _check(self._lib.kfp_mlp_layer_shape(self._h, int(layer), ctypes.byref(i), ctypes.byref(o)))
        return i.value, o.value

    def forward(self, X, out=None, stream=None):
        import torch

        n_out = self.shape(self.layers() - 1)[1]
        B = check_mlp_io(self.shape(0)[0], n_out, X, out=out)
        Y = out if out is not None else torch.empty((B, n_out), dtype=torch.float32, device=X.device)
        _check(self._lib.kfp_mlp_forward(self._h, int(B), _fptr(X, torch.float32),
                                         _fptr(Y, torch.float32), _stream(stream)))
        return Y

    def backward(self, X, T, stream=None):
        import torch

        check_mlp_io(self.shape(0)[0], self.shape(self.layers() - 1)[1], X, T)
        loss = ctypes.c_double()
        _check(self._lib.kfp_mlp_backward(self._h, int(X.shape[0]), _fptr(X, torch.float32),
                                          _fptr(T, torch.float32), ctypes.byref(loss),
                                          _stream(stream)))
        return loss.value

    def adam(self, lr, stream=None):
        _check(self._lib.kfp_mlp_adam(self._h, float(lr), _stream(stream)))

    def train_step(self, X, T, lr, stream=None):
        import torch

        check_mlp_io(self.shape(0)[0], self.shape(self.layers() - 1)[1], X, T)
        loss = ctypes.c_double()
        _check(self._lib.kfp_mlp_train_step(self._h, int(X.shape[0]), _fptr(X, torch.float32),
                                            _fptr(T, torch.float32), float(lr),
                                            ctypes.byref(loss), _stream(stream)))
        return loss.value

    def get(self, layer, which, stream=None):
        """which: 'W', 'b', 'dW', 'db' -> float32 GPU tensor."""
        import torch

        code = {"W": 0, "b": 1, "dW": 2, "db": 3}[which]
        i, o = self.shape(layer)
        shape = (o, i) if code in (0, 2) else (o,)
        buf = torch.empty(shape, dtype=torch.float32, device="cuda")
        _check(self._lib.kfp_mlp_param(self._h, int(layer), code, 0, _fptr(buf), _stream(stream)))
        return buf

    def set(self, layer, which, value, stream=None):
        import torch

        code = {"W": 0, "b": 1}[which]
        i, o = self.shape(layer)
        _expect(value, (o, i) if code == 0 else (o,), which)
        v = value.to(device="cuda", dtype=torch.float32).contiguous()
        _check(self._lib.kfp_mlp_param(self._h, int(layer), code, 1, _fptr(v), _stream(stream)))
        torch.cuda.current_stream().synchronize()


def cast_f64_f32(src, dst, base=None, stream=None):
    """dst = (float)(src - base); base None for none."""
    import torch

    lib = _mlp_sigs(load_library())
    n = int(src.numel())
    if dst.numel() != n or (base is not None and base.numel() != n):
        raise KfpError(KFP_EINVAL, f"cast_f64_f32: sizes differ ({n}, {dst.numel()})")
    bp = None if base is None else _fptr(base, torch.float64)
    _check(lib.kfp_cast_f64_f32(_fptr(src, torch.float64), bp, _fptr(dst, torch.float32), n,
                                _stream(stream)))


def axpy_f32(x, y, alpha, stream=None):
    """y += alpha * x (FP32, same size, in place)."""
    import torch

    lib = _mlp_sigs(load_library())
    if x.numel() != y.numel():
        raise KfpError(KFP_EINVAL, "axpy_f32: sizes differ")
    _check(lib.kfp_axpy_f32(_fptr(x, torch.float32), _fptr(y, torch.float32), float(alpha),
                            int(y.numel()), _stream(stream)))


def mul_f32(a, y, stream=None):
    """y *= a element-wise (FP32, same size, in place)."""
    import torch

    lib = _mlp_sigs(load_library())
    if a.numel() != y.numel():
        raise KfpError(KFP_EINVAL, "mul_f32: sizes differ")
    _check(lib.kfp_mul_f32(_fptr(a, torch.float32), _fptr(y, torch.float32), int(y.numel()),
                           _stream(stream)))


def column_stats(X, floor=1e-6, stream=None):
    import torch

    lib = _mlp_sigs(load_library())
    rows, cols = X.shape
    mean = torch.empty(cols, dtype=torch.float32, device=X.device)
    std = torch.empty(cols, dtype=torch.float32, device=X.device)
    _check(lib.kfp_column_stats(_fptr(X, torch.float32), int(rows), int(cols), float(floor),
                                _fptr(mean), _fptr(std), _stream(stream)))
    return mean, std


def standardize(X, mean, std, stream=None):
    import torch

    lib = _mlp_sigs(load_library())
    rows, cols = X.shape
    _expect(mean, (cols,), "mean")
    _expect(std, (cols,), "std")
    _check(lib.kfp_standardize(_fptr(X, torch.float32), int(rows), int(cols), _fptr(mean),
                               _fptr(std), _stream(stream)))


def destandardize(Y, mean, std, out=None, base=None, stream=None):
    """lam = base + mean + std * Y in FP64 (base [rows][cols] FP64 or None)."""
    import torch

    lib = _mlp_sigs(load_library())
    rows, cols = Y.shape
    _expect(mean, (cols,), "mean")
    _expect(std, (cols,), "std")
    if out is not None and out.numel() != rows * cols:
        raise ValueError("destandardize: out has the wrong size")
    lam = out if out is not None else torch.empty((rows, cols), dtype=torch.float64, device=Y.device)
    if base is not None and base.numel() != rows * cols:
        raise KfpError(KFP_EINVAL, "destandardize: base has the wrong size")
    bp = None if base is None else _fptr(base, torch.float64)
    _check(lib.kfp_destandardize(_fptr(Y, torch.float32), int(rows), int(cols), _fptr(mean),
                                 _fptr(std), bp, _fptr(lam, torch.float64), _stream(stream)))
    return lam


def _modes_arg(modes):
    m = [int(x) for x in modes]
    if not 1 <= len(m) <= 8:
        raise ValueError("1..8 x frequencies")
    return len(m), (ctypes.c_int32 * len(m))(*m)


def trace_modes(lam, modes, out=None, stream=None):
    """x-Fourier coefficients of trace rows: lam [..., nx] FP64 ->
    [..., 2 len(modes)] with (cos, sin) coefficient pairs per frequency."""
    import torch

    lib = _mlp_sigs(load_library())
    if lam.dim() < 1:
        raise ValueError("trace_modes: lam needs an x dimension")
    nx = int(lam.shape[-1])
    rows = lam.numel() // max(nx, 1)
    nm, arr = _modes_arg(modes)
    shape = tuple(lam.shape[:-1]) + (2 * nm,)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=lam.device)
    _expect(out, shape, "out")
    _check(lib.kfp_trace_modes(_fptr(lam, torch.float64), int(rows), nx, nm, arr,
                               _fptr(out, torch.float64), _stream(stream)))
    return out


def trace_synth(coef, modes, nt, nx, out=None, stream=None):
    """Traces [planes][nt][nx] FP64 from x-Fourier coefficients
    coef [planes][ntc][2 len(modes)], linear in time between coefficient
    levels (see kfp_trace_synth)."""
    import torch

    lib = _mlp_sigs(load_library())
    nm, arr = _modes_arg(modes)
    if coef.dim() != 3 or coef.shape[2] != 2 * nm:
        raise ValueError(f"trace_synth: coef must be [planes][ntc][{2 * nm}]")
    planes, ntc = int(coef.shape[0]), int(coef.shape[1])
    shape = (planes, int(nt), int(nx))
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=coef.device)
    _expect(out, shape, "out")
    _check(lib.kfp_trace_synth(_fptr(coef, torch.float64), planes, ntc, nm, arr, int(nt),
                               int(nx), _fptr(out, torch.float64), _stream(stream)))
    return out

"""CPU FP64 oracle for the SWR method on the Kolmogorov equation.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark are the only callers.  The GPU library never
imports, links or runs anything in this directory, and this directory never
imports the GPU library.

The arithmetic lives in ``kfp_oracle.c`` (plain C, FP64, Thomas with
divisions); this module compiles it with gcc and wraps it with ctypes.  The
MLP oracle (forward, backward, Adam) is ``oracle.mlp`` in plain numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kfp_oracle.c")
_LIB = os.path.join(_HERE, "libkfp_oracle.so")

DIRICHLET = 0
ROBIN = 1
FD = 0   # finite differences in v, IMEX step (the default discretisation)
FEM = 1  # linear finite elements, diffusion then transport (Section 6.2 as printed)

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/libkfp_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.{os.getpid()}.tmp"  # one per process: concurrent builds do not mix
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.c_int
        lib.oracle_thomas.argtypes = [I, D, D, D, D, D]
        lib.oracle_transport.argtypes = [I, I, I, ctypes.c_double, D, D]
        lib.oracle_mono_solve.argtypes = [I, I, I, ctypes.c_double, D, D, D, D]
        lib.oracle_partition.argtypes = [I, I, I, ctypes.POINTER(I), ctypes.POINTER(I)]
        lib.oracle_swr_solve.argtypes = [
            I, I, I, ctypes.c_double, D, D, D, I, I, I, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, I, D, D, D, ctypes.POINTER(I), D, D,
        ]
        lib.oracle_swr_solve_ordered.argtypes = [
            I, I, I, ctypes.c_double, D, D, D, I, I, I, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, I, D, I, D, D, ctypes.POINTER(I), D, D,
        ]
        lib.oracle_swr_solve_scheme.argtypes = [
            I, I, I, ctypes.c_double, D, D, D, I, I, I, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, I, D, I, I, D, D, ctypes.POINTER(I), D, D,
        ]
        lib.oracle_fem_mono_solve.argtypes = [I, I, I, ctypes.c_double, D, D, D, D]
        lib.oracle_u0_guess.argtypes = [I, I, I, D, I, I, I, ctypes.c_double, ctypes.c_double, D]
        for fn in ("oracle_thomas", "oracle_transport", "oracle_mono_solve",
                   "oracle_partition", "oracle_swr_solve", "oracle_swr_solve_ordered",
                   "oracle_swr_solve_scheme", "oracle_fem_mono_solve", "oracle_u0_guess"):
            getattr(lib, fn).restype = I
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    """Set the OpenMP thread count the oracle uses (its column loops)."""
    os.environ["OMP_NUM_THREADS"] = str(int(n))
    try:
        omp = ctypes.CDLL("libgomp.so.1")
        omp.omp_set_num_threads(int(n))
    except OSError:
        pass


def thomas(lo, di, up, rhs):
    """Plain Thomas solve of one tridiagonal system (row i: lo x_{i-1} + di x_i + up x_{i+1})."""
    lo, di, up, rhs = map(_f64, (lo, di, up, rhs))
    x = np.empty_like(rhs)
    if _load().oracle_thomas(len(rhs), _p(lo), _p(di), _p(up), _p(rhs), _p(x)):
        raise ValueError("bad system")
    return x


def transport(U, T, nt):
    """One upwind x-transport step (eqs. (6.4)/(6.5)) of a full [nv+1][nx] field."""
    U = _f64(U)
    nv, nx = U.shape[0] - 1, U.shape[1]
    out = np.empty_like(U)
    if _load().oracle_transport(nx, nv, nt, float(T), _p(U), _p(out)):
        raise ValueError("bad transport arguments")
    return out


def partition(nv, J, o):
    """Subdomain node ranges [a_j, b_j] (eq. (6.6) generalised to J pieces)."""
    a = (ctypes.c_int * J)()
    b = (ctypes.c_int * J)()
    if _load().oracle_partition(nv, J, o, a, b):
        raise ValueError("invalid partition")
    return list(a), list(b)


def mono_solve(u0, f, T, nt, s=None, scheme=FD):
    """Monodomain discrete solution at t = T, [nv+1][nx].  scheme FD: finite
    differences with zero values at v = +-1; FEM: linear finite elements with
    Neumann ends, diffusion then transport (Section 6.2)."""
    u0, f = _f64(u0), _f64(f)
    nv, nx = u0.shape[0] - 1, u0.shape[1]
    s = None if s is None else _f64(s)
    uT = np.empty_like(u0)
    fn = _load().oracle_fem_mono_solve if scheme == FEM else _load().oracle_mono_solve
    if scheme not in (FD, FEM):
        raise ValueError("unknown scheme")
    if fn(nx, nv, nt, float(T), _p(u0), _p(f), _p(s), _p(uT)):
        raise ValueError("invalid arguments")
    return uT


class SWRResult:
    def __init__(self, uT, lam, iters, res_hist, ovl_hist, status):
        self.uT = uT
        self.lam = lam
        self.iters = iters
        self.res_hist = res_hist
        self.ovl_hist = ovl_hist
        self.status = status

    @property
    def residual(self):
        return float(self.res_hist[-1])


def swr_solve(u0, f, T, nt, J, overlap, transmission, p=0.0, tol=1e-12, max_iter=100,
              lambda_init=None, s=None, q=None, order=0, scheme=FD):
    """SWR (Section 6.3).  Returns SWRResult.  q: second Robin parameter of
    OSWR(p,q); None for q = p.  order: 0 parallel (the Jacobi Remark after
    (6.12)), 1 multiplicative in red-black order (even subdomains, then odd
    ones with the traces the even ones just sent; for two subdomains the
    serial form (6.8)-(6.11)).  scheme: FD or FEM (see mono_solve); with FEM
    the iterates, traces and residual are those of the diffusion stage."""
    u0, f = _f64(u0), _f64(f)
    nv, nx = u0.shape[0] - 1, u0.shape[1]
    s = None if s is None else _f64(s)
    nI = J - 1
    lam_out = np.zeros((max(2 * nI, 1), nt, nx))
    li = None if lambda_init is None else _f64(lambda_init)
    if li is not None and li.shape != (2 * nI, nt, nx):
        raise ValueError("lambda_init shape")
    uT = np.empty_like(u0)
    hist = np.zeros(max_iter)
    ovl = np.zeros(max_iter)
    it = ctypes.c_int(0)
    st = _load().oracle_swr_solve_scheme(nx, nv, nt, float(T), _p(u0), _p(f), _p(s), J,
                                         overlap, int(transmission), float(p),
                                         float(p if q is None else q), float(tol), max_iter,
                                         _p(li), int(order), int(scheme), _p(uT), _p(lam_out),
                                         ctypes.byref(it), _p(hist), _p(ovl))
    if st == 1:
        raise ValueError("invalid arguments")
    k = it.value
    return SWRResult(uT, lam_out[: 2 * nI], k, hist[:k].copy(), ovl[:k].copy(), st)


def swr_solve_windows(u0, f, T, nt, J, overlap, transmission, p=0.0, tol=1e-12, max_iter=100,
                      n_windows=1, s=None, q=None, guess=False, order=0, scheme=FD):
    """SWR on time windows: [0, T] is cut into n_windows windows of whole
    steps (window w takes steps floor(w nt / W) .. floor((w+1) nt / W) - 1),
    and each is solved by swr_solve to the tolerance, starting from the glued
    iterate at the end of the window before (window 0 from u0), with zero
    initial traces or (guess) the u0_guess extension of that start state.
    Returns (uT, per-window iteration counts, per-window statuses)."""
    u0 = _f64(u0)
    dt = T / nt
    start = u0
    iters, status = [], []
    for w in range(n_windows):
        n0 = w * nt // n_windows
        n1 = (w + 1) * nt // n_windows
        ntw = n1 - n0
        sw = None if s is None else _f64(s)[n0:n1 + 1]
        lam0 = u0_guess(start, ntw, J, overlap, transmission, p, q) if guess and J > 1 else None
        r = swr_solve(start, f, ntw * dt, ntw, J, overlap, transmission, p=p, tol=tol,
                      max_iter=max_iter, lambda_init=lam0, s=sw, q=q, order=order,
                      scheme=scheme)
        iters.append(r.iters)
        status.append(r.status)
        start = r.uT
    return start, iters, status


def u0_guess(u0, nt, J, overlap, transmission, p=0.0, q=None):
    """Initial traces lambda^0(n) = Q(u0) at each interface node, for every n."""
    u0 = _f64(u0)
    nv, nx = u0.shape[0] - 1, u0.shape[1]
    lam = np.zeros((2 * (J - 1), nt, nx))
    if _load().oracle_u0_guess(nx, nv, nt, _p(u0), J, overlap, int(transmission), float(p),
                               float(p if q is None else q), _p(lam)):
        raise ValueError("invalid arguments")
    return lam

"""CPU tests of the library's host side: exported symbols, argument validation
(every EINVAL path returns before any device call) and the elimination tables
of the segment-partitioned tridiagonal solve."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1306_4596_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.lib_path()):
        pytest.skip("libkfpswr not built")
    return binding.load_library()


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(kfp_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert {"kfp_mono_solve", "kfp_swr_solve", "kfp_swr_batch"} <= names
    for name in sorted(names):
        assert hasattr(lib, name), name


G = binding.Grid
FAKE = ctypes.c_void_p(256)  # never dereferenced: validation fails first


def swr(lib, g, J=2, o=2, tr=1, p=4.0, tol=1e-10, max_iter=10, u0=FAKE, f=FAKE, uT=FAKE):
    return lib.kfp_swr_solve(ctypes.byref(g), u0, f, None, J, o, tr, p, tol, max_iter, None, uT,
                             None, None, None)


@pytest.mark.parametrize("kw,frag", [
    (dict(g=G(1, 64, 10, 0.1)), "nx"),
    (dict(g=G(64, 2, 10, 0.1)), "nv"),
    (dict(g=G(64, 64, 0, 0.1)), "nt"),
    (dict(g=G(64, 64, 10, -1.0)), "T"),
    (dict(g=G(1024, 64, 10, 1.0)), "CFL"),
    (dict(J=3), "nv % J"),
    (dict(J=16, o=3), "nv/J"),
    (dict(tr=0, o=0), "overlap"),
    (dict(p=0.0), "p must be"),
    (dict(p=-1.0), "p must be"),
    (dict(tr=7), "transmission"),
    (dict(tol=0.0), "tol"),
    (dict(max_iter=0), "max_iter"),
    (dict(u0=None), "non-NULL"),
    (dict(uT=None), "non-NULL"),
])
def test_swr_invalid_arguments(lib, kw, frag):
    args = dict(g=G(64, 64, 10, 0.1))
    args.update(kw)
    st = swr(lib, **args)
    assert st == binding.KFP_EINVAL
    assert frag in lib.kfp_last_error().decode()


def test_mono_and_batch_invalid_arguments(lib):
    g = G(64, 64, 10, 0.1)
    assert lib.kfp_mono_solve(ctypes.byref(g), None, FAKE, None, FAKE, None) == binding.KFP_EINVAL
    bad = G(64, 64, 10, 100.0)
    assert lib.kfp_mono_solve(ctypes.byref(bad), FAKE, FAKE, None, FAKE, None) == binding.KFP_EINVAL
    inst = (binding.Instance * 1)()
    inst[0].g = G(64, 64, 10, 0.1)
    inst[0].J, inst[0].overlap, inst[0].tr, inst[0].p = 3, 2, 1, 4.0
    assert lib.kfp_swr_batch(1, inst, 1e-10, 10, None, None) == binding.KFP_EINVAL
    assert "instance 0" in lib.kfp_last_error().decode()
    assert lib.kfp_swr_batch(0, inst, 1e-10, 10, None, None) == binding.KFP_EINVAL
    assert lib.kfp_set_config(3, 8, 1) == binding.KFP_EINVAL
    assert lib.kfp_set_config(4, 24, 40) == binding.KFP_EINVAL
    assert lib.kfp_set_config(4, 48, 4) == binding.KFP_EINVAL
    assert lib.kfp_bw_probe(FAKE, FAKE, 10, None) == binding.KFP_EINVAL
    # the tile probe: unbuilt shapes, null pointers and empty widths are refused
    assert lib.kfp_tile_probe(FAKE, FAKE, FAKE, 10, 64, 8, 16, None) == binding.KFP_EINVAL
    assert lib.kfp_tile_probe(None, FAKE, FAKE, 10, 64, 8, 17, None) == binding.KFP_EINVAL
    assert lib.kfp_tile_probe(FAKE, FAKE, FAKE, 10, 0, 8, 17, None) == binding.KFP_EINVAL
    assert lib.kfp_tile_probe(FAKE, FAKE, FAKE, -1, 64, 8, 17, None) == binding.KFP_EINVAL
    assert lib.kfp_tile_probe(FAKE, FAKE, FAKE, 8 * 17 * 65536, 64, 8, 17, None) == binding.KFP_EINVAL


def test_static_mono_validation(lib):
    """The no-allocation monodomain entry point validates like kfp_mono_solve
    and rejects a grid whose state and tables exceed its static workspace,
    before any device call."""
    g = G(64, 64, 10, 0.1)
    assert lib.kfp_mono_solve_static(ctypes.byref(g), None, FAKE, None, FAKE,
                                     None) == binding.KFP_EINVAL
    bad = G(64, 64, 10, 100.0)
    assert lib.kfp_mono_solve_static(ctypes.byref(bad), FAKE, FAKE, None, FAKE,
                                     None) == binding.KFP_EINVAL
    big = G(4096, 4096, 100, 0.01)  # 2 x 4095 x 4096 doubles of state: 268 MB
    assert lib.kfp_mono_solve_static(ctypes.byref(big), FAKE, FAKE, None, FAKE,
                                     None) == binding.KFP_EINVAL
    assert "static workspace" in lib.kfp_last_error().decode()


def test_subdomain_rows(lib):
    r = ctypes.c_int64()
    g = G(1024, 1024, 2000, 0.5)
    assert lib.kfp_subdomain_rows(ctypes.byref(g), 8, 2, 1, ctypes.byref(r)) == 0
    assert r.value == 1023 + 7 * 3  # (nv - 1) + (J - 1)(o + 1) for Robin
    assert lib.kfp_subdomain_rows(ctypes.byref(g), 8, 2, 0, ctypes.byref(r)) == 0
    assert r.value == 1023 + 7 * 1  # (nv - 1) + (J - 1)(o - 1) for Dirichlet
    # no overlap (Robin only): the shared node is a row of both neighbours
    assert lib.kfp_subdomain_rows(ctypes.byref(g), 8, 0, 1, ctypes.byref(r)) == 0
    assert r.value == 1023 + 7


def get_tables(lib, nx, nv, nt, T, J, o, tr, p, waves):
    g = G(nx, nv, nt, T)
    r = ctypes.c_int64()
    assert lib.kfp_subdomain_rows(ctypes.byref(g), J, o, tr, ctypes.byref(r)) == 0
    rows = np.zeros((r.value, 6))
    mat = np.zeros((r.value, 3))
    info = np.zeros((J, 8), dtype=np.int32)
    segs = np.zeros(J * (waves + 1), dtype=np.int32)
    reds = np.zeros((J * waves, 5))
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    lib.kfp_debug_tables.argtypes = [ctypes.POINTER(G), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
    st = lib.kfp_debug_tables(ctypes.byref(g), J, o, tr, p, waves, P(info), P(rows), P(segs),
                              P(reds), P(mat))
    assert st == 0, lib.kfp_last_error()
    return info, rows, segs, reds, mat


def paper_matrix(nv, nt, T, lo_node, n, lo_kind, hi_kind, p):
    """Tridiagonal matrix of one subdomain's unknown rows from Section 6.2/6.3:
    implicit-Euler diffusion rows [-r, 1+2r, -r]; a Robin row (q - d/dv) at a
    lower interface, (p + d/dv) at an upper one (q = p); without overlap the
    shared node's half-cell row: [1+2r+2 dt p/h_v, -2r] (times 2 dt/h_v, the
    balance of the half cell with the Robin flux)."""
    hv = 2.0 / nv
    r = (T / nt) / hv ** 2
    hc = 2.0 * (T / nt) / hv
    A = np.zeros((n, n))
    for k in range(n):
        A[k, k] = 1 + 2 * r
        if k > 0:
            A[k, k - 1] = -r
        if k < n - 1:
            A[k, k + 1] = -r
    if lo_kind == 2:
        A[0, :] = 0
        A[0, 0], A[0, 1] = p + 1 / hv, -1 / hv
    if hi_kind == 2:
        A[n - 1, :] = 0
        A[n - 1, n - 2], A[n - 1, n - 1] = -1 / hv, p + 1 / hv
    if lo_kind == 3:
        A[0, :] = 0
        A[0, 0], A[0, 1] = 1 + 2 * r + hc * p, -2 * r
    if hi_kind == 3:
        A[n - 1, :] = 0
        A[n - 1, n - 2], A[n - 1, n - 1] = -2 * r, 1 + 2 * r + hc * p
    return A


def emulate_partitioned_solve(rows, segs, reds, P, d):
    """The kernel's algorithm, step by step: local Thomas per segment with the
    precomputed factors, reduced separator system, spike correction."""
    n = len(d)
    ys, first, last, sep = [], np.zeros(P), np.zeros(P), np.zeros(P)
    for w in range(P):
        s0, s1 = segs[w], segs[w + 1]
        blk = (s1 - s0 - 1) if w < P - 1 else (s1 - s0)
        y = np.zeros(blk)
        for k in range(blk):
            fa, fb = rows[s0 + k, 1], rows[s0 + k, 2]
            y[k] = d[s0 + k] * fa if k == 0 else fb * y[k - 1] + d[s0 + k] * fa
        for k in range(blk - 1, -1, -1):
            if k < blk - 1:
                y[k] = rows[s0 + k, 3] * y[k + 1] + y[k]
        ys.append(y)
        first[w], last[w] = y[0], y[-1]
        if w < P - 1:
            sep[w] = d[s1 - 1]
    xi = np.zeros(max(P - 1, 0))
    z = np.zeros(max(P - 1, 0))
    for s in range(P - 1):
        ra, rc, g1, g2, h = reds[s]
        D = sep[s] - ra * last[s] - rc * first[s + 1]
        z[s] = D * g1 if s == 0 else g2 * z[s - 1] + D * g1
    for s in range(P - 2, -1, -1):
        xi[s] = z[s] if s == P - 2 else reds[s, 4] * xi[s + 1] + z[s]
    x = np.zeros(n)
    for w in range(P):
        s0 = segs[w]
        xlo = xi[w - 1] if w >= 1 else 0.0
        xhi = xi[w] if w < P - 1 else 0.0
        y = ys[w]
        for k in range(len(y)):
            x[s0 + k] = y[k] - rows[s0 + k, 4] * xlo - rows[s0 + k, 5] * xhi
        if w < P - 1:
            x[s0 + len(y)] = xhi
    return x


@pytest.mark.parametrize("nx,nv,nt,T,J,o,tr,p", [
    (64, 64, 200, 0.1, 2, 4, 0, 0.0),
    (1024, 1024, 2000, 0.5, 8, 2, 1, 4.0),
    (256, 256, 512, 0.5, 4, 2, 1, 4.0),
    (128, 1024, 512, 0.25, 2, 2, 1, 4.0),
    (64, 48, 100, 0.1, 3, 5, 1, 0.7),
    (16, 16, 10, 0.1, 1, 0, 0, 0.0),
    (128, 128, 100, 0.1, 4, 0, 1, 3.0),
])
@pytest.mark.parametrize("waves", [1, 2, 4, 8, 16])
def test_partitioned_tables_solve_the_paper_matrix(lib, nx, nv, nt, T, J, o, tr, p, waves):
    info, rows, segs, reds, mat = get_tables(lib, nx, nv, nt, T, J, o, tr, p, waves)
    rng = np.random.default_rng(waves + 10 * J)
    hx, hv, dt = 1.0 / nx, 2.0 / nv, T / nt
    red_off = 0
    for j in range(J):
        n, row_off, g_lo, P, lo_kind, hi_kind, tab, seg = info[j]
        A = paper_matrix(nv, nt, T, g_lo, n, lo_kind, hi_kind, p)
        sub = mat[tab:tab + n]
        assert np.array_equal(np.diag(A), sub[:, 1])
        assert np.array_equal(np.diag(A, -1), sub[1:, 0])
        assert np.array_equal(np.diag(A, 1), sub[:-1, 2])
        nu = (-1.0 + (g_lo + np.arange(n)) * hv) * dt / hx
        assert np.allclose(rows[tab:tab + n, 0], nu, rtol=0, atol=1e-15)
        assert P == max(1, min(waves, n // 2))
        sg = segs[seg:seg + P + 1] - 0
        assert sg[0] == 0 and sg[-1] == n and np.all(np.diff(sg) >= (1 if P == 1 else 1))
        d = rng.standard_normal(n)
        x = emulate_partitioned_solve(rows[tab:tab + n], sg, reds[red_off:red_off + P - 1], P, d)
        ref = np.linalg.solve(A, d)
        assert np.allclose(x, ref, rtol=0, atol=1e-12 * np.abs(ref).max()), (j, P)
        red_off += P - 1


def test_bench_counters_only_for_the_measured_kernel(tmp_path, monkeypatch):
    """The roofline's counter figures (HBM traffic, VALU busy) are reported
    only for the launch configuration and kernel sources the counters were
    taken on; the compulsory-bytes model stays below the one-step streaming
    bytes and grows with the steps of a launch."""
    import importlib
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    bench = importlib.import_module("bench")
    assert not bench.counters_valid((1, 2, 3, 1, 0))
    cfg = bench.COUNTERS["config"]
    if cfg is not None:
        assert bench.counters_valid(cfg)
        # a copy of the tree with one changed source byte reports nothing
        for rel in bench.COUNTERS["sha256"]:
            src = os.path.join(root, rel)
            dst = tmp_path / rel
            dst.parent.mkdir(parents=True, exist_ok=True)
            dst.write_bytes(open(src, "rb").read() + b" ")
        monkeypatch.setattr(bench, "ROOT", str(tmp_path))
        assert not bench.counters_valid(cfg)
    rows = (bench.NV - 1) + (bench.J - 1) * (bench.OVERLAP + 1)
    b12 = bench.compulsory_bytes_per_launch(rows, 12)
    # state in and out plus the source: 24 bytes per cell once per launch
    assert b12 > 24.0 * bench.NX * rows
    assert b12 < 24.0 * bench.NX * rows * 12
    assert bench.compulsory_bytes_per_launch(rows, 16) > b12


def test_ordering_launch_and_window_arguments(lib):
    """Validation of the ordering, lane-group launch and time-window entry
    points (no device call is reached)."""
    assert lib.kfp_set_ordering(2) == binding.KFP_EINVAL
    assert lib.kfp_set_ordering(-1) == binding.KFP_EINVAL
    assert lib.kfp_set_ordering(0) == 0
    # lane groups: compiled set, halo must leave columns (2 * steps * groups < 64)
    assert lib.kfp_set_launch(8, 2, 33, 6) == 0
    assert lib.kfp_set_launch(8, 2, 33, 16) == binding.KFP_EINVAL
    assert lib.kfp_set_launch(8, 4, 33, 8) == binding.KFP_EINVAL
    assert lib.kfp_set_launch(8, 3, 33, 4) == binding.KFP_EINVAL
    assert lib.kfp_set_launch(4, 2, 8, 0) == binding.KFP_EINVAL  # one-step kernel: groups 1
    assert lib.kfp_set_launch(0, 1, 0, 0) == 0
    g = G(64, 64, 10, 0.1)
    its = (ctypes.c_int32 * 4)()

    def win(n_windows, guess=0, J=2, o=2, tr=1, u0=FAKE):
        return lib.kfp_swr_solve_windows(ctypes.byref(g), u0, FAKE, None, J, o, tr, 4.0, 4.0,
                                         1e-10, 10, n_windows, guess, FAKE, its, None, None)
    assert win(0) == binding.KFP_EINVAL and "n_windows" in lib.kfp_last_error().decode()
    assert win(11) == binding.KFP_EINVAL
    assert win(2, guess=2) == binding.KFP_EINVAL
    assert win(2, u0=None) == binding.KFP_EINVAL
    assert win(2, J=3) == binding.KFP_EINVAL and "nv % J" in lib.kfp_last_error().decode()
    assert win(2, tr=0, o=0) == binding.KFP_EINVAL


@pytest.mark.parametrize("J,o,tr,p", [(1, 0, 0, 0.0), (2, 2, 1, 4.0), (3, 0, 1, 3.0),
                                      (3, 3, 0, 0.0), (4, 1, 1, 2.5)])
def test_fem_rows_are_the_element_matrices(lib, J, o, tr, p):
    """With the finite-element scheme each subdomain's matrix is dt/h_v times
    (M/dt + S) of its own elements (Simpson-integrated basis functions), with
    dt/h_v p (q) on a Robin end row and the fixed nodes of a classical
    interface removed; v = -1 and v = +1 are unknown rows (Neumann)."""
    nx, nv, nt, T = 32, 48, 40, 0.5
    assert lib.kfp_set_scheme(1) == 0
    try:
        info, rows, segs, reds, mat = get_tables(lib, nx, nv, nt, T, J, o, tr, p, 4)
        r = ctypes.c_int64()
        g = G(nx, nv, nt, T)
        assert lib.kfp_subdomain_rows(ctypes.byref(g), J, o, tr, ctypes.byref(r)) == 0
    finally:
        assert lib.kfp_set_scheme(0) == 0
    assert r.value == nv + 1 + (J - 1) * (o + 1 if tr == 1 else o - 1)
    import oracle
    from tests import dense_ref
    a, b = oracle.partition(nv, J, o)
    hv, dt = 2.0 / nv, T / nt
    for j in range(J):
        n, row_off, g_lo, P, lo_kind, hi_kind, tab, seg = info[j]
        M, S = dense_ref.fem_matrices(nv, a[j], b[j])
        A = (M / dt + S) * (dt / hv)
        lo = a[j] if (j == 0 or tr == 1) else a[j] + 1
        hi = b[j] if (j == J - 1 or tr == 1) else b[j] - 1
        assert (g_lo, n) == (lo, hi - lo + 1)
        if tr == 1 and j > 0:
            A[a[j], a[j]] += dt / hv * p
        if tr == 1 and j < J - 1:
            A[b[j], b[j]] += dt / hv * p
        A = A[lo:hi + 1, lo:hi + 1]
        sub = mat[tab:tab + n]
        assert np.allclose(sub[:, 1], np.diag(A), rtol=1e-13, atol=0)
        assert np.allclose(sub[1:, 0], np.diag(A, -1), rtol=1e-13, atol=0)
        assert np.allclose(sub[:-1, 2], np.diag(A, 1), rtol=1e-13, atol=0)


def test_fem_scheme_arguments(lib):
    assert lib.kfp_set_scheme(2) == binding.KFP_EINVAL
    assert lib.kfp_set_scheme(-1) == binding.KFP_EINVAL
    assert lib.kfp_set_scheme(1) == 0
    try:
        # one subdomain of 4097 rows: no march configuration holds it
        g = G(64, 4096, 64, 0.5)
        st = lib.kfp_swr_solve(ctypes.byref(g), FAKE, FAKE, None, 1, 0, 0, 0.0, 1e-10, 5, None,
                               FAKE, None, None, None)
        assert st == binding.KFP_EINVAL
        assert "finite-element scheme" in lib.kfp_last_error().decode()
    finally:
        assert lib.kfp_set_scheme(0) == 0


def test_fem_batch_rejects_tall_instances(lib):
    """A batch instance whose subdomains no march configuration holds is
    rejected under the finite-element scheme, before any device call."""
    inst = (binding.Instance * 2)()
    inst[0].g = G(64, 64, 10, 0.1)
    inst[0].J, inst[0].overlap, inst[0].tr, inst[0].p = 2, 2, 1, 4.0
    inst[1].g = G(64, 4096, 10, 0.1)
    inst[1].J, inst[1].overlap, inst[1].tr, inst[1].p = 1, 0, 0, 0.0
    for i in range(2):
        inst[i].u0 = inst[i].f = inst[i].uT = FAKE
    assert lib.kfp_set_scheme(1) == 0
    try:
        assert lib.kfp_swr_batch(2, inst, 1e-10, 10, None, None) == binding.KFP_EINVAL
        msg = lib.kfp_last_error().decode()
        assert "instance 1" in msg and "finite-element" in msg
    finally:
        assert lib.kfp_set_scheme(0) == 0


def test_fem_rejects_r_below_one_sixth(lib):
    """With finite elements the end-node mismatch equals the overlap maximum
    (6.12) only while the element matrix is an M-matrix (r >= 1/6): SWR
    solves below that are rejected; the monodomain solve is not affected."""
    assert lib.kfp_set_scheme(1) == 0
    try:
        # r = (T/nt) / (2/nv)^2 = (0.01/100) / (1/32)^2 = 0.1024 < 1/6
        g = G(64, 64, 100, 0.01)
        st = lib.kfp_swr_solve(ctypes.byref(g), FAKE, FAKE, None, 2, 2, 1, 4.0, 1e-10, 5, None,
                               FAKE, None, None, None)
        assert st == binding.KFP_EINVAL
        assert "1/6" in lib.kfp_last_error().decode()
        r = ctypes.c_int64()
        assert lib.kfp_subdomain_rows(ctypes.byref(g), 1, 0, 0, ctypes.byref(r)) == 0
    finally:
        assert lib.kfp_set_scheme(0) == 0
    # finite differences: the same shape is accepted as far as validation goes
    g = G(64, 64, 100, 0.01)
    r = ctypes.c_int64()
    assert lib.kfp_subdomain_rows(ctypes.byref(g), 2, 2, 1, ctypes.byref(r)) == 0


def _meta(*shape, dtype=None):
    import torch

    return torch.empty(shape, dtype=dtype or torch.float64, device="meta")


@pytest.mark.parametrize("call,frag", [
    ("mono_f", "f has shape"),
    ("mono_out", "out has shape"),
    ("swr_f", "f has shape"),
    ("swr_lam", "lambda_init has shape"),
    ("swr_lam_J1", "J < 2"),
    ("win_f", "f has shape"),
    ("batch_lam", "lambda_init has shape"),
])
def test_binding_rejects_mis_sized_tensors(call, frag):
    """Every tensor is checked against its documented shape before any
    pointer reaches the library (the kernels would read or write past a
    short buffer): f and uT like u0, lambda_init [2(J-1)][nt][nx]."""
    u0 = _meta(65, 64)
    nt = 10
    with pytest.raises(ValueError, match=frag):
        if call == "mono_f":
            binding.mono_solve(u0, _meta(65, 63), 0.1, nt)
        elif call == "mono_out":
            binding.mono_solve(u0, _meta(65, 64), 0.1, nt, out=_meta(64, 64))
        elif call == "swr_f":
            binding.swr_solve(u0, _meta(64, 64), 0.1, nt, 2, 2, 1, p=4.0)
        elif call == "swr_lam":
            binding.swr_solve(u0, _meta(65, 64), 0.1, nt, 2, 2, 1, p=4.0,
                              lambda_init=_meta(2, nt - 1, 64))
        elif call == "swr_lam_J1":
            binding.swr_solve(u0, _meta(65, 64), 0.1, nt, 1, 0, 0, lambda_init=_meta(0, nt, 64))
        elif call == "win_f":
            binding.swr_solve_windows(u0, _meta(65, 32), 0.1, nt, 2, 2, 1, p=4.0, n_windows=2)
        elif call == "batch_lam":
            binding.swr_batch([dict(u0=u0, f=_meta(65, 64), T=0.1, nt=nt, J=4, overlap=2, tr=1,
                                    p=4.0, lambda_init=_meta(2, nt, 64))])


def test_network_io_shapes():
    """X is [B][n_in], T and out [B][n_out]: anything else is rejected before
    the GEMM kernels see the pointers."""
    import torch

    f32 = torch.float32
    assert binding.check_mlp_io(64, 10, _meta(8, 64, dtype=f32), _meta(8, 10, dtype=f32)) == 8
    for X, T, out, frag in [
        (_meta(8, 63, dtype=f32), None, None, "X has shape"),
        (_meta(8, 64, dtype=f32), _meta(8, 11, dtype=f32), None, "T has shape"),
        (_meta(8, 64, dtype=f32), _meta(7, 10, dtype=f32), None, "T has shape"),
        (_meta(8, 64, dtype=f32), None, _meta(8, 9, dtype=f32), "out has shape"),
        (_meta(64, dtype=f32), None, None, "X must be"),
        (_meta(0, 64, dtype=f32), None, None, "empty"),
    ]:
        with pytest.raises(ValueError, match=frag):
            binding.check_mlp_io(64, 10, X, T, out)


def test_trace_mode_arguments(lib):
    """The x-Fourier trace helpers reject bad frequencies and sizes before
    any device call."""
    i32 = ctypes.c_int32
    lib.kfp_trace_modes.argtypes = [ctypes.c_void_p, ctypes.c_int64, i32, i32,
                                    ctypes.POINTER(i32), ctypes.c_void_p, ctypes.c_void_p]
    lib.kfp_trace_synth.argtypes = [ctypes.c_void_p, i32, i32, i32, ctypes.POINTER(i32), i32,
                                    i32, ctypes.c_void_p, ctypes.c_void_p]
    m = (i32 * 4)(1, 2, 3, 4)
    assert lib.kfp_trace_modes(FAKE, 4, 8, 4, m, FAKE, None) == binding.KFP_EINVAL  # 2*4 >= 8
    assert "frequency" in lib.kfp_last_error().decode()
    assert lib.kfp_trace_modes(FAKE, 4, 64, 0, m, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_modes(FAKE, 4, 64, 9, m, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_modes(FAKE, 4, 64, 4, None, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_modes(None, 4, 64, 4, m, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_modes(FAKE, -1, 64, 4, m, FAKE, None) == binding.KFP_EINVAL
    z = (i32 * 1)(0)
    assert lib.kfp_trace_modes(FAKE, 4, 64, 1, z, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_synth(FAKE, 0, 4, 4, m, 8, 64, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_synth(FAKE, 2, 0, 4, m, 8, 64, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_synth(FAKE, 2, 4, 4, m, 0, 64, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_synth(FAKE, 2, 4, 4, m, 8, 6, FAKE, None) == binding.KFP_EINVAL
    assert lib.kfp_trace_synth(None, 2, 4, 4, m, 8, 64, FAKE, None) == binding.KFP_EINVAL


def test_windows_with_initial_traces_arguments(lib):
    """kfp_swr_solve_windows_init validates like kfp_swr_solve_windows and
    needs the initial traces when there are interfaces."""
    g = G(64, 64, 10, 0.1)
    its = (ctypes.c_int32 * 4)()

    def win(n_windows, lam=FAKE, J=2, u0=FAKE):
        return lib.kfp_swr_solve_windows_init(ctypes.byref(g), u0, FAKE, None, J, 2, 1, 4.0, 4.0,
                                              1e-10, 10, n_windows, lam, FAKE, its, None, None)
    assert win(2, lam=None) == binding.KFP_EINVAL
    assert "lambda_init" in lib.kfp_last_error().decode()
    assert win(0) == binding.KFP_EINVAL and "n_windows" in lib.kfp_last_error().decode()
    assert win(11) == binding.KFP_EINVAL
    assert win(2, u0=None) == binding.KFP_EINVAL

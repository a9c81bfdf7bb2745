"""GPU parity of the finite-element scheme (Section 6.2 as printed: linear
elements with the consistent mass matrix, Neumann ends, diffusion then
transport) through the C ABI against the CPU oracle.

Tolerances as in test_gpu_parity: relative L2 <= 1e-12 for fixed iteration
counts and the monodomain march (the same arithmetic up to rounding order),
<= 1e-10 for converged solves.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1306_4596_amd as kfp  # noqa: E402
from paper_1306_4596_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

D, R, FEM = kfp.DIRICHLET, kfp.ROBIN, oracle.FEM


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _fem():
    kfp.set_config(0)
    kfp.set_pipeline(-1)
    kfp.set_ordering(kfp.PARALLEL)
    kfp.set_scheme(kfp.FEM)
    yield
    kfp.set_scheme(kfp.FD)
    kfp.set_config(0)
    kfp.set_pipeline(-1)
    kfp.set_ordering(kfp.PARALLEL)
    os.environ.pop("KFP_NO_GRAPH", None)


@pytest.mark.parametrize("nx,nv,nt,T,cfg", [(64, 64, 40, 0.1, None), (5, 8, 3, 0.3, None),
                                            (100, 40, 37, 0.2, (4, 8, 1)),
                                            (40, 16, 11, 0.2, (4, 8, 8)),
                                            (70, 62, 20, 0.2, (4, 8, 6, 2)),
                                            (30, 300, 25, 0.3, None)])
def test_fem_mono_matches_oracle(nx, nv, nt, T, cfg):
    print(f"fem mono nx={nx} nv={nv} nt={nt} cfg={cfg}", flush=True)
    u0, f = inputs.random_fields(nx + nv, nx, nv)
    s = 1.0 + 0.5 * np.sin(np.arange(nt + 1))
    ref = oracle.mono_solve(u0, f, T, nt, s, scheme=FEM)
    if cfg:
        kfp.set_config(*cfg[:3], groups=cfg[3] if len(cfg) > 3 else 1)
    out = host(kfp.mono_solve(dev(u0), dev(f), T, nt, s=s))
    assert rel(out, ref) <= 1e-12


CASES = [
    # nx, nv, nt, T, J, o, tr, p, q
    (64, 64, 40, 0.1, 2, 4, D, 0.0, None),
    (64, 64, 30, 0.3, 4, 2, R, 4.0, None),
    (100, 96, 20, 0.2, 3, 3, R, 2.5, 0.9),
    (70, 120, 16, 0.2, 8, 1, D, 0.0, None),
    (72, 128, 24, 0.25, 4, 5, R, 8.0, None),
    (64, 64, 30, 0.2, 2, 0, R, 3.0, None),
    (48, 96, 20, 0.2, 4, 0, R, 2.0, 5.0),
    (40, 64, 20, 0.2, 2, 1, R, 6.0, None),
]


@pytest.mark.parametrize("case", CASES)
def test_fem_fixed_iterations_match_oracle(case):
    nx, nv, nt, T, J, o, tr, p, q = case
    print(f"fem swr fixed K case={case}", flush=True)
    u0, f = inputs.random_fields(7, nx, nv)
    s = 1.0 + 0.3 * np.cos(np.arange(nt + 1))
    lam0 = inputs.random_traces(11, J, nt, nx)
    K = 4
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-300, max_iter=K,
                           lambda_init=lam0, s=s, scheme=FEM)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-300,
                                max_iter=K, lambda_init=dev(lam0), s=s, want_lambda=True)
    assert st.iters == K
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("case", CASES)
def test_fem_converged_matches_oracle_and_monodomain(case):
    nx, nv, nt, T, J, o, tr, p, q = case
    print(f"fem swr converged case={case}", flush=True)
    u0, f = inputs.random_fields(3, nx, nv)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-12, max_iter=2000,
                           scheme=FEM)
    uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-12,
                              max_iter=2000)
    assert st.iters == ref.iters
    assert rel(host(uT), ref.uT) <= 1e-10
    mono = oracle.mono_solve(u0, f, T, nt, scheme=FEM)
    assert rel(host(uT), mono) <= 1e-10


CONFIGS = [
    # nx, nv, J, (waves, seg, steps[, groups])
    (40, 56, 2, (1, 32, 1)),
    (40, 64, 2, (2, 24, 3)),
    (40, 64, 2, (4, 12, 5)),
    (40, 64, 4, (8, 4, 2)),
    (40, 96, 3, (8, 6, 7)),
    (40, 128, 2, (16, 6, 4)),
    (40, 64, 2, (4, 8, 3, 2)),
    (50, 256, 2, (8, 17, 4, 2)),
    (40, 768, 3, (8, 24, 6, 2)),
    (40, 1024, 2, (8, 33, 2, 4)),
]


@pytest.mark.parametrize("case", CONFIGS)
@pytest.mark.parametrize("tr", [D, R])
def test_fem_launch_configurations(case, tr):
    """Segments of every length and count (a padded last segment, lane
    groups, fewer segments than the workgroup holds, the reduced system in
    registers and in LDS) against the oracle, three iterations."""
    nx, nv, J, cfg = case
    nt, T, o = 12, 0.1, 2
    print(f"fem config nx={nx} nv={nv} J={J} cfg={cfg} tr={tr}", flush=True)
    u0, f = inputs.random_fields(31 + nv + J, nx, nv)
    p = 4.0 if tr == R else 0.0
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3, scheme=FEM)
    kfp.set_config(*cfg[:3], groups=cfg[3] if len(cfg) > 3 else 1)
    got = kfp.get_launch(nx, nv, nt, T, J, o, tr)
    assert got[2] == cfg[2] and got[0] == cfg[0]
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


RB_CASES = [
    # nx, nv, nt, T, J, o, tr, p, q, cfg
    (72, 64, 30, 0.2, 2, 4, D, 0.0, None, None),
    (72, 64, 30, 0.2, 2, 2, R, 4.0, None, (4, 8, 5)),
    (80, 96, 24, 0.2, 3, 2, R, 11.0, 2.5, None),
    (64, 64, 24, 0.2, 4, 0, R, 3.0, None, (2, 12, 3)),
]


@pytest.mark.parametrize("case", RB_CASES)
def test_fem_red_black_matches_oracle(case):
    nx, nv, nt, T, J, o, tr, p, q, cfg = case
    print(f"fem red-black case={case}", flush=True)
    u0, f = inputs.random_fields(70 + J, nx, nv)
    lam0 = inputs.random_traces(71, J, nt, nx)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-300, max_iter=4,
                           lambda_init=lam0, order=1, scheme=FEM)
    if cfg:
        kfp.set_config(*cfg)
    kfp.set_ordering(kfp.RED_BLACK)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-300,
                                max_iter=4, lambda_init=dev(lam0), want_lambda=True)
    assert st.iters == 4
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-11, max_iter=400, order=1,
                           scheme=FEM)
    for inflight in (0, 4):  # staggered half-sweeps, then overlapped ones
        kfp.set_pipeline(inflight)
        uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                                  max_iter=400)
        assert st.iters == ref.iters, inflight
        assert rel(host(uT), ref.uT) <= 1e-10


@pytest.mark.parametrize("inflight", [2, 5])
def test_fem_overlapped_iterations_equal_plain(inflight):
    nx, nv, nt, T, J, o = 64, 64, 40, 0.2, 4, 2
    u0, f = inputs.random_fields(5, nx, nv)
    kfp.set_config(4, 8, 4)
    kfp.set_pipeline(0)
    a, _, sa = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, R, p=4.0, tol=1e-11, max_iter=300)
    kfp.set_pipeline(inflight)
    b, _, sb = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, R, p=4.0, tol=1e-11, max_iter=300)
    assert sa.iters == sb.iters
    assert torch.equal(a, b)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, R, p=4.0, tol=1e-11, max_iter=300, scheme=FEM)
    assert sa.iters == ref.iters and rel(host(a), ref.uT) <= 1e-10


@pytest.mark.parametrize("case", [(48, 64, 37, 0.2, 2, 2, R, 4.0, None, 4, False, 0),
                                  (40, 64, 12, 0.1, 2, 4, D, 0.0, None, 3, True, 0),
                                  (64, 96, 30, 0.2, 3, 0, R, 5.0, None, 3, True, 1)])
def test_fem_time_windows_match_oracle(case):
    nx, nv, nt, T, J, o, tr, p, q, W, guess, order = case
    print(f"fem windows case={case}", flush=True)
    u0, f = inputs.random_fields(90 + W, nx, nv)
    s = 1.0 + 0.3 * np.cos(np.arange(nt + 1))
    kfp.set_ordering(order)
    ref, rit, _ = oracle.swr_solve_windows(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                                           max_iter=400, n_windows=W, s=s, guess=guess,
                                           order=order, scheme=FEM)
    uT, its, st = kfp.swr_solve_windows(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                                        max_iter=400, n_windows=W, s=s, guess=guess)
    assert its == rit and st.iters == sum(rit)
    assert rel(host(uT), ref) <= 1e-10
    m = oracle.mono_solve(u0, f, T, nt, s, scheme=FEM)
    assert rel(host(uT), m) <= 1e-9


@pytest.mark.parametrize("order", [0, 1])
def test_fem_batch_matches_single_solves_and_oracle(order):
    specs = [
        (64, 64, 40, 0.2, 2, 2, R, 4.0),
        (128, 32, 40, 0.1, 4, 2, R, 2.0),
        (96, 128, 40, 0.3, 8, 2, D, 0.0),
        (64, 256, 40, 0.2, 2, 3, R, 8.0),
        (64, 64, 40, 0.15, 1, 0, R, 1.0),
        (48, 64, 30, 0.2, 4, 0, R, 3.0),
    ]
    kfp.set_ordering(order)
    kfp.set_config(8, 17, 4, groups=2)  # one configuration for the batch and the singles
    insts, singles = [], []
    for i, (nx, nv, nt, T, J, o, tr, p) in enumerate(specs):
        u0, f = inputs.random_fields(100 + i, nx, nv)
        insts.append(dict(u0=dev(u0), f=dev(f), T=T, nt=nt, J=J, overlap=o, tr=tr, p=p))
        singles.append(kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-11,
                                     max_iter=400))
    out, rc = kfp.swr_batch(insts, tol=1e-11, max_iter=400)
    assert rc == 0
    for (uT, _, st), (suT, _, sst) in zip(out, singles):
        assert st.iters == sst.iters
        assert torch.equal(uT, suT)
    for i, ((nx, nv, nt, T, J, o, tr, p), (uT, _, st)) in enumerate(zip(specs, out)):
        u0, f = inputs.random_fields(100 + i, nx, nv)
        ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-11, max_iter=400,
                               order=order if J > 1 else 0, scheme=FEM)
        assert st.iters == ref.iters, i
        assert rel(host(uT), ref.uT) <= 1e-10, i


def test_fem_rejects_the_one_step_kernel():
    kfp.set_config(4, 16, 0)
    u0, f = inputs.random_fields(1, 32, 32)
    with pytest.raises(kfp.KfpError, match="finite-element"):
        kfp.swr_solve(dev(u0), dev(f), 0.1, 10, 2, 2, R, p=4.0, tol=1e-10, max_iter=5)


def test_fem_benchmark_shape_fixed_iterations():
    """1024 x 1024, J = 8, overlap 2, Robin p = 8 (the benchmark's shape) on a
    short window, with the launch configuration the library picks: two
    iterations against the oracle."""
    nx = nv = 1024
    nt, T = 16, 0.004
    u0, f = inputs.random_fields(0, nx, nv)
    print("fem benchmark shape oracle ...", flush=True)
    ref = oracle.swr_solve(u0, f, T, nt, 8, 2, R, p=8.0, tol=1e-300, max_iter=2, scheme=FEM)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 8, 2, R, p=8.0, tol=1e-300, max_iter=2,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12


def test_fem_scheme_is_a_setting():
    """FD and FEM give different answers on the same input; switching back
    restores the finite-difference result exactly."""
    nx, nv, nt, T = 48, 64, 20, 0.2
    u0, f = inputs.random_fields(2, nx, nv)
    a, _, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 2, R, p=4.0, tol=1e-11, max_iter=200)
    kfp.set_scheme(kfp.FD)
    b, _, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 2, R, p=4.0, tol=1e-11, max_iter=200)
    ref = oracle.swr_solve(u0, f, T, nt, 2, 2, R, p=4.0, tol=1e-11, max_iter=200)
    assert rel(host(b), ref.uT) <= 1e-10
    assert rel(host(a), host(b)) > 1e-6

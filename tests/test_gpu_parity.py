"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerance: relative L2 <= 1e-10 in FP64 for converged solves (the target the
method is held to) and <= 1e-12 for fixed iteration counts and the
monodomain march, where both sides run the same arithmetic up to the
rounding order of the Thomas elimination (divisions on the CPU, precomputed
reciprocals and a segment partition on the GPU).
"""
import ctypes
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1306_4596_amd as kfp  # noqa: E402
from paper_1306_4596_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

D, R = kfp.DIRICHLET, kfp.ROBIN


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _auto_config():
    kfp.set_config(0)
    kfp.set_pipeline(-1)
    kfp.set_ordering(kfp.PARALLEL)
    yield
    kfp.set_config(0)
    kfp.set_pipeline(-1)
    kfp.set_ordering(kfp.PARALLEL)
    os.environ.pop("KFP_NO_GRAPH", None)


# ------------------------------------------------------------ monodomain ---
@pytest.mark.parametrize("nx,nv,nt,T", [(64, 64, 200, 0.1), (100, 40, 37, 0.2), (5, 8, 3, 0.3),
                                        (130, 300, 50, 0.3)])
def test_mono_matches_oracle(nx, nv, nt, T):
    print(f"mono nx={nx} nv={nv} nt={nt}", flush=True)
    u0, f = inputs.random_fields(nx + nv, nx, nv)
    s = 1.0 + 0.5 * np.sin(np.arange(nt + 1))
    ref = oracle.mono_solve(u0, f, T, nt, s)
    out = host(kfp.mono_solve(dev(u0), dev(f), T, nt, s=s))
    torch.cuda.synchronize()
    assert rel(out, ref) <= 1e-12
    assert np.all(out[0] == 0) and np.all(out[-1] == 0)


def test_mono_manufactured_cfg0():
    nx = nv = 64
    nt, T = 200, 0.1
    u0, f, s, ex = inputs.manufactured(nx, nv, nt, T)
    ref = oracle.mono_solve(u0, f, T, nt, s)
    out = host(kfp.mono_solve(dev(u0), dev(f), T, nt, s=s))
    assert rel(out, ref) <= 1e-12
    assert np.abs(out - ex(T)).max() / np.abs(ex(T)).max() < 2e-2


# ---------------------------------------------------------------- SWR -------
CASES = [
    # nx, nv, nt, T, J, o, tr, p
    (64, 64, 200, 0.1, 2, 4, D, 0.0),
    (64, 64, 60, 0.3, 4, 2, R, 4.0),
    (100, 96, 40, 0.2, 3, 3, R, 2.5),
    (70, 120, 30, 0.2, 8, 1, D, 0.0),
    (200, 128, 64, 0.25, 4, 5, R, 8.0),
]


@pytest.mark.parametrize("case", CASES)
def test_swr_fixed_iterations_match_oracle(case):
    nx, nv, nt, T, J, o, tr, p = case
    print(f"swr fixed K case={case}", flush=True)
    u0, f = inputs.random_fields(7, nx, nv)
    K = 4
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-300, max_iter=K)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-300, max_iter=K,
                                want_lambda=True)
    assert st.iters == K
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("case", CASES)
def test_swr_converged_matches_oracle_and_monodomain(case):
    nx, nv, nt, T, J, o, tr, p = case
    print(f"swr converged case={case}", flush=True)
    u0, f = inputs.random_fields(3, nx, nv)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-12, max_iter=2000)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-12, max_iter=2000,
                                want_lambda=True)
    assert st.iters == ref.iters
    assert rel(host(uT), ref.uT) <= 1e-10
    mono = oracle.mono_solve(u0, f, T, nt)
    assert rel(host(uT), mono) <= 1e-10


def test_cfg0_manufactured_swr():
    nx = nv = 64
    nt, T = 200, 0.1
    u0, f, s, _ = inputs.manufactured(nx, nv, nt, T)
    ref = oracle.swr_solve(u0, f, T, nt, 2, 4, D, tol=1e-12, max_iter=500, s=s)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 4, D, tol=1e-12, max_iter=500, s=s,
                                want_lambda=True)
    assert st.iters == ref.iters and st.residual < 1e-12
    assert rel(host(uT), ref.uT) <= 1e-10
    assert rel(host(lam), ref.lam) <= 1e-10


def test_error_equation_and_initial_guess():
    nx, nv, nt, T, J, o = 64, 64, 50, 0.25, 2, 3
    z = np.zeros((nv + 1, nx))
    lam0 = inputs.random_traces(1, J, nt, nx)
    ref = oracle.swr_solve(z, z, T, nt, J, o, R, p=4.0, tol=1e-300, max_iter=6, lambda_init=lam0)
    uT, lam, st = kfp.swr_solve(dev(z), dev(z), T, nt, J, o, R, p=4.0, tol=1e-300, max_iter=6,
                                lambda_init=dev(lam0), want_lambda=True)
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=0)


@pytest.mark.parametrize("pq", [(11.0, 2.5), (0.8, 6.0)])
def test_two_sided_robin_matches_oracle(pq):
    """OSWR(p,q) of Section 6.4.2: fixed iterations and converged solves."""
    p, q = pq
    nx, nv, nt, T, J, o = 80, 96, 40, 0.25, 4, 2
    u0, f = inputs.random_fields(31, nx, nv)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, R, p=p, q=q, tol=1e-300, max_iter=4)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, R, p=p, q=q, tol=1e-300,
                                max_iter=4, want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, R, p=p, q=q, tol=1e-11, max_iter=1000)
    uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, R, p=p, q=q, tol=1e-11,
                              max_iter=1000)
    assert st.iters == ref.iters
    assert rel(host(uT), ref.uT) <= 1e-10
    assert rel(host(uT), oracle.mono_solve(u0, f, T, nt)) <= 1e-10
    g = host(kfp.u0_guess(dev(u0), nt, J, o, R, p=p, q=q))
    assert rel(g, oracle.u0_guess(u0, nt, J, o, R, p=p, q=q)) <= 1e-14
    # the batch takes q per instance
    out, rc = kfp.swr_batch([dict(u0=dev(u0), f=dev(f), T=T, nt=nt, J=J, overlap=o, tr=R, p=p,
                                  q=q)], tol=1e-11, max_iter=1000)
    assert rc == 0 and out[0][2].iters == ref.iters
    assert rel(host(out[0][0]), ref.uT) <= 1e-10


def test_u0_guess_matches_oracle():
    nx, nv, nt = 80, 64, 20
    u0, _ = inputs.random_fields(4, nx, nv)
    for tr, p in ((D, 0.0), (R, 3.0)):
        ref = oracle.u0_guess(u0, nt, 4, 2, tr, p=p)
        out = host(kfp.u0_guess(dev(u0), nt, 4, 2, tr, p=p))
        assert rel(out, ref) <= 1e-14


def test_nonfinite_guess_restarts_from_zero():
    nx, nv, nt, T = 64, 32, 20, 0.2
    u0, f = inputs.random_fields(2, nx, nv)
    bad = np.zeros((2, nt, nx))
    bad[0, 3, 5] = np.nan
    uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 2, R, p=4.0, tol=1e-11, max_iter=300,
                              lambda_init=dev(bad))
    assert st.restarted
    ref = oracle.swr_solve(u0, f, T, nt, 2, 2, R, p=4.0, tol=1e-11, max_iter=300)
    assert st.iters == ref.iters
    assert rel(host(uT), ref.uT) <= 1e-10


def test_resume_from_returned_traces():
    nx, nv, nt, T = 64, 64, 30, 0.2
    u0, f = inputs.random_fields(6, nx, nv)
    a, la, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=4.0, tol=1e-300, max_iter=6,
                             want_lambda=True)
    b1, lb1, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=4.0, tol=1e-300, max_iter=3,
                               want_lambda=True)
    b2, lb2, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=4.0, tol=1e-300, max_iter=3,
                               lambda_init=lb1, want_lambda=True)
    assert torch.equal(a, b2) and torch.equal(la, lb2)


def test_cached_plan_takes_each_calls_time_step():
    """Solves of one shape with different T share the cached buffers; each
    must still use its own dt (also after u0_guess, which takes any valid T)."""
    nx, nv, nt, J, o = 64, 64, 40, 4, 2
    u0, f = inputs.random_fields(13, nx, nv)
    kfp.u0_guess(dev(u0), nt, J, o, R, p=4.0)
    for T in (0.2, 0.05, 0.2):
        ref = oracle.swr_solve(u0, f, T, nt, J, o, R, p=4.0, tol=1e-300, max_iter=3)
        uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, R, p=4.0, tol=1e-300,
                                    max_iter=3, want_lambda=True)
        assert rel(host(uT), ref.uT) <= 1e-12, T
        assert rel(host(lam), ref.lam) <= 1e-12, T


def test_max_iter_returns_last_iterate():
    nx, nv, nt, T = 64, 64, 30, 0.2
    u0, f = inputs.random_fields(6, nx, nv)
    with pytest.raises(kfp.KfpError):
        kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 2, D, tol=1e-14, max_iter=1, raise_noconv=True)
    uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 2, D, tol=1e-14, max_iter=1)
    ref = oracle.swr_solve(u0, f, T, nt, 2, 2, D, tol=1e-14, max_iter=1)
    assert st.iters == 1 and ref.status == 4
    assert rel(host(uT), ref.uT) <= 1e-12


# ------------------------------------------------- launch configurations ----
CONFIGS = [(1, 0, 0), (1, 64, 0), (2, 0, 0), (2, 48, 0), (4, 16, 0), (4, 32, 0), (8, 8, 0),
           (8, 0, 0), (16, 8, 0), (16, 0, 0),
           # register march kernel: (waves, seg_max, steps per launch)
           (4, 24, 1), (8, 10, 1), (16, 6, 1),
           (4, 24, 2), (4, 24, 8), (8, 10, 4), (8, 10, 7), (16, 8, 8), (16, 6, 16),
           (8, 24, 12), (4, 32, 5), (16, 12, 9)]


@pytest.mark.parametrize("waves,seg,steps", CONFIGS)
@pytest.mark.parametrize("tr", [D, R])
def test_every_launch_configuration_agrees(waves, seg, steps, tr):
    nx, nv, nt, T, J, o = 96, 128, 24, 0.2, 2, 2
    print(f"config waves={waves} seg={seg} steps={steps} tr={tr}", flush=True)
    u0, f = inputs.random_fields(9, nx, nv)
    p = 4.0 if tr == R else 0.0
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3)
    kfp.set_config(waves, seg, steps)
    got = kfp.get_config(nx, nv, nt, T, J, o, tr)
    # a forced register segment too short for the subdomain is widened to the
    # next compiled size (or the memory-staged variant)
    assert got[0] == waves and got[2] == steps and (got[1] == 0 or got[1] >= seg)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


# J = 4 on 64 v-cells: about 19 rows per subdomain, interior subdomains with
# transmission rows at both ends; single- and two-wave register segments
CONFIGS_J4 = [(1, 0, 0), (2, 0, 0), (4, 8, 0), (1, 24, 1), (1, 24, 8), (1, 32, 3), (2, 12, 4),
              (2, 16, 8), (4, 6, 2), (4, 8, 8), (8, 4, 1), (8, 4, 8)]


@pytest.mark.parametrize("waves,seg,steps", CONFIGS_J4)
@pytest.mark.parametrize("tr", [D, R])
def test_launch_configurations_interior_subdomains(waves, seg, steps, tr):
    nx, nv, nt, T, J, o = 80, 64, 20, 0.2, 4, 2
    print(f"config J=4 waves={waves} seg={seg} steps={steps} tr={tr}", flush=True)
    u0, f = inputs.random_fields(14, nx, nv)
    p = 4.0 if tr == R else 0.0
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3)
    kfp.set_config(waves, seg, steps)
    got = kfp.get_config(nx, nv, nt, T, J, o, tr)
    assert got[0] == waves and got[2] == steps
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


# Lane groups: each wavefront holds `groups` segments of 64/groups columns.
# The shapes fill some wavefronts, leave one with a single active group and
# others idle, give every group count a tall case that only it holds, and
# end the x-range in a ragged tile (or a grid narrower than one tile).
GROUP_CASES = [
    # nx, nv, J, (waves, seg, steps, groups)
    (40, 64, 2, (4, 8, 1, 2)),
    (40, 96, 3, (4, 8, 5, 2)),
    (40, 64, 4, (4, 8, 15, 2)),
    (50, 256, 2, (8, 17, 4, 2)),
    (40, 512, 2, (8, 17, 8, 2)),
    (40, 768, 3, (8, 24, 6, 2)),
    (40, 1024, 2, (8, 33, 4, 2)),
    (40, 1024, 2, (8, 33, 2, 4)),
    (30, 2048, 2, (8, 33, 3, 4)),
    (5, 512, 2, (8, 17, 4, 2)),
]


@pytest.mark.parametrize("case", GROUP_CASES)
@pytest.mark.parametrize("tr", [D, R])
def test_lane_group_configurations(case, tr):
    nx, nv, J, (waves, seg, steps, groups) = case
    nt, T, o = 12, 0.1, 2
    print(f"lane groups nx={nx} nv={nv} J={J} cfg={(waves, seg, steps, groups)} tr={tr}",
          flush=True)
    u0, f = inputs.random_fields(31 + nv + J, nx, nv)
    p = 4.0 if tr == R else 0.0
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3)
    kfp.set_config(waves, seg, steps, groups=groups)
    assert kfp.get_launch(nx, nv, nt, T, J, o, tr) == (waves, seg, steps, groups)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-300, max_iter=3,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


def test_lane_groups_mono_and_default_choice():
    """The monodomain march in lane groups, and the built-in choice for a
    subdomain taller than eight wavefronts of register segments."""
    nx, nv, nt, T = 70, 64, 20, 0.2
    u0, f = inputs.random_fields(77, nx, nv)
    ref = oracle.mono_solve(u0, f, T, nt)
    kfp.set_config(4, 8, 6, groups=2)
    assert rel(host(kfp.mono_solve(dev(u0), dev(f), T, nt)), ref) <= 1e-12
    kfp.set_config(0)
    got = kfp.get_launch(1024, 1024, 40, 0.01, 2, 2, R)
    assert got[3] >= 2 and got[2] >= 1, got
    got = kfp.get_launch(64, 2048, 40, 0.01, 2, 2, R)
    assert got[3] == 4 and got[2] >= 1, got


@pytest.mark.parametrize("steps", [0, 1, 8])
def test_mono_multi_step_and_tiny_grids(steps):
    """The march kernel on grids narrower than its tiles (lanes wrap around
    the periodic x-range) and with a window shorter than one launch."""
    for nx, nv, nt, T in ((5, 8, 3, 0.3), (40, 16, 11, 0.2), (64, 64, 20, 0.2)):
        u0, f = inputs.random_fields(nx + 3 * nv, nx, nv)
        ref = oracle.mono_solve(u0, f, T, nt)
        kfp.set_config(4, 8, steps) if nv // 2 - 1 <= 32 else kfp.set_config(0)
        out = host(kfp.mono_solve(dev(u0), dev(f), T, nt))
        assert rel(out, ref) <= 1e-12, (nx, nv, nt, steps)


def test_graph_and_direct_launch_agree_and_are_deterministic():
    nx, nv, nt, T = 128, 128, 40, 0.2
    u0, f = inputs.random_fields(12, nx, nv)
    a, la, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=2.0, tol=1e-300, max_iter=5,
                             want_lambda=True)
    b, lb, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=2.0, tol=1e-300, max_iter=5,
                             want_lambda=True)
    os.environ["KFP_NO_GRAPH"] = "1"
    c, lc, _ = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=2.0, tol=1e-300, max_iter=5,
                             want_lambda=True)
    assert torch.equal(a, b) and torch.equal(la, lb)
    assert torch.equal(a, c) and torch.equal(la, lc)


# ------------------------------------------------------ no overlap (L = 0) --
# The shared interface node is a half-cell row of both neighbours; traces
# (p + q) u - lambda.  One-step kernels (memory-staged and register
# segments), march kernels with and without lane groups.
NONOVL_CONFIGS = [None, (1, 0, 0), (2, 16, 0), (4, 8, 0), (8, 0, 0), (4, 24, 1), (4, 24, 8),
                  (8, 10, 4), (4, 8, 5, 2)]


@pytest.mark.parametrize("cfg", NONOVL_CONFIGS)
@pytest.mark.parametrize("J,p,q", [(2, 4.0, None), (4, 2.0, 5.0)])
def test_without_overlap_matches_oracle(cfg, J, p, q):
    nx, nv, nt, T = 72, 64, 24, 0.2
    print(f"no overlap cfg={cfg} J={J} p={p} q={q}", flush=True)
    u0, f = inputs.random_fields(40 + J, nx, nv)
    ref = oracle.swr_solve(u0, f, T, nt, J, 0, R, p=p, q=q, tol=1e-300, max_iter=3)
    if cfg:
        kfp.set_config(*cfg)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, 0, R, p=p, q=q, tol=1e-300,
                                max_iter=3, want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


def test_without_overlap_converges_overlapped_and_batched():
    nx, nv, nt, T = 64, 64, 40, 0.2
    u0, f = inputs.random_fields(41, nx, nv)
    ref = oracle.swr_solve(u0, f, T, nt, 4, 0, R, p=3.0, tol=1e-11, max_iter=400)
    assert ref.status == 0
    runs = []
    for mode in (0, 3):
        kfp.set_pipeline(mode)
        uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 0, R, p=3.0, tol=1e-11,
                                    max_iter=400, want_lambda=True)
        assert st.iters == ref.iters
        assert rel(host(uT), ref.uT) <= 1e-10
        runs.append((uT, lam))
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    kfp.set_pipeline(-1)
    # a batch mixing overlapping and non-overlapping instances equals the singles
    specs = [(64, 64, 40, 0.2, 4, 0, 3.0), (96, 128, 40, 0.2, 2, 2, 4.0),
             (64, 128, 40, 0.1, 2, 0, 6.0)]
    insts, singles = [], []
    kfp.set_config(4, 8, 4)  # one configuration (widened per shape) for both
    for i, (nx_, nv_, nt_, T_, J_, o_, p_) in enumerate(specs):
        a, b = inputs.random_fields(50 + i, nx_, nv_)
        insts.append(dict(u0=dev(a), f=dev(b), T=T_, nt=nt_, J=J_, overlap=o_, tr=R, p=p_))
        singles.append(kfp.swr_solve(dev(a), dev(b), T_, nt_, J_, o_, R, p=p_, tol=1e-11,
                                     max_iter=400))
    out, rc = kfp.swr_batch(insts, tol=1e-11, max_iter=400)
    assert rc == 0
    for (uT, _, st), (ruT, _, rst) in zip(out, singles):
        assert st.iters == rst.iters and torch.equal(uT, ruT)


# ------------------------------------------------ red-black (multiplicative) --
RB_CASES = [
    # nx, nv, nt, T, J, o, tr, p, q, cfg
    (72, 64, 30, 0.2, 2, 4, D, 0.0, None, None),
    (72, 64, 30, 0.2, 2, 2, R, 4.0, None, (4, 8, 5)),
    (80, 96, 24, 0.2, 3, 2, R, 11.0, 2.5, None),
    (64, 64, 24, 0.2, 4, 0, R, 3.0, None, (2, 12, 3)),
    (50, 128, 20, 0.2, 4, 3, D, 0.0, None, (8, 4, 1)),
    (40, 512, 12, 0.1, 2, 2, R, 4.0, None, (8, 17, 4, 2)),
]


@pytest.mark.parametrize("case", RB_CASES)
def test_red_black_matches_oracle(case):
    nx, nv, nt, T, J, o, tr, p, q, cfg = case
    print(f"red-black case={case}", flush=True)
    u0, f = inputs.random_fields(70 + J, nx, nv)
    lam0 = inputs.random_traces(71, J, nt, nx)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-300, max_iter=4,
                           lambda_init=lam0, order=1)
    if cfg:
        kfp.set_config(*cfg)
    kfp.set_ordering(kfp.RED_BLACK)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-300,
                                max_iter=4, lambda_init=dev(lam0), want_lambda=True)
    assert st.iters == 4
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)
    # converged: same count as the oracle, the monodomain solution
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-11, max_iter=400, order=1)
    uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                              max_iter=400)
    assert st.iters == ref.iters
    assert rel(host(uT), ref.uT) <= 1e-10
    os.environ["KFP_NO_GRAPH"] = "1"
    uT2, _, st2 = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                                max_iter=400)
    assert st2.iters == st.iters and torch.equal(uT, uT2)


@pytest.mark.parametrize("case", [RB_CASES[0], RB_CASES[2], RB_CASES[3], RB_CASES[5]])
@pytest.mark.parametrize("inflight", [2, 5])
def test_red_black_overlapped_half_sweeps_equal_staggered(case, inflight):
    """Red-black half-sweeps overlapped in time (slots of one colour each)
    reproduce the staggered red-black iteration bit for bit: iterate,
    traces, count and residual history."""
    nx, nv, nt, T, J, o, tr, p, q, cfg = case
    print(f"red-black overlapped case={case} inflight={inflight}", flush=True)
    u0, f = inputs.random_fields(72 + J, nx, nv)
    if cfg:
        kfp.set_config(*cfg)
    kfp.set_ordering(kfp.RED_BLACK)
    runs = []
    for mode in (0, inflight):
        kfp.set_pipeline(mode)
        runs.append(kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                                  max_iter=400, want_lambda=True))
    (a, la, sa), (b, lb, sb) = runs
    assert sa.iters == sb.iters and sa.residual < 1e-11
    assert torch.equal(a, b) and torch.equal(la, lb)
    assert np.array_equal(sa.res_history, sb.res_history)
    kfp.set_pipeline(inflight)
    c, lc, sc = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-300,
                              max_iter=3, want_lambda=True)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-300, max_iter=3, order=1)
    assert sc.iters == 3
    assert rel(host(c), ref.uT) <= 1e-12 and rel(host(lc), ref.lam) <= 1e-12


def test_red_black_batch_matches_single_solves():
    """Red-black order in a batch of uneven instances (several launch
    classes, odd and even J, with and without overlap) equals the single
    red-black solves bit for bit, and the oracle to the tolerance."""
    specs = [(64, 64, 40, 0.2, 2, 2, R, 4.0), (128, 32, 40, 0.1, 4, 2, R, 2.0),
             (96, 96, 40, 0.3, 3, 2, D, 0.0), (64, 256, 40, 0.2, 2, 0, R, 8.0),
             (80, 512, 30, 0.2, 2, 2, R, 4.0), (64, 64, 40, 0.15, 1, 0, R, 1.0)]
    kfp.set_ordering(kfp.RED_BLACK)
    kfp.set_pipeline(0)  # the single solves in the staggered form
    insts, singles = [], []
    for i, (nx, nv, nt, T, J, o, tr, p) in enumerate(specs):
        u0, f = inputs.random_fields(120 + i, nx, nv)
        insts.append(dict(u0=dev(u0), f=dev(f), T=T, nt=nt, J=J, overlap=o, tr=tr, p=p,
                          want_lambda=True))
        singles.append(kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-11,
                                     max_iter=400, want_lambda=True))
    out, rc = kfp.swr_batch(insts, tol=1e-11, max_iter=400)
    assert rc == 0
    for i, ((uT, lam, st), (ruT, rlam, rst)) in enumerate(zip(out, singles)):
        assert st.iters == rst.iters, i
        assert torch.equal(uT, ruT), i
        if lam is not None:
            assert torch.equal(lam, rlam), i
        nx, nv, nt, T, J, o, tr, p = specs[i]
        u0, f = inputs.random_fields(120 + i, nx, nv)
        ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-11, max_iter=400, order=1)
        assert st.iters == ref.iters and rel(host(uT), ref.uT) <= 1e-10, i


@pytest.mark.parametrize("inflight", [0, 4])
def test_red_black_guess_restart_and_iteration_cap(inflight):
    """Red-black order, staggered and overlapped: a non-finite initial guess
    restarts from zero traces; a solve stopped by max_iter returns that
    iterate (the oracle's after the same count) and reports no convergence."""
    nx, nv, nt, T, J = 64, 32, 40, 0.2, 4
    u0, f = inputs.random_fields(2, nx, nv)
    kfp.set_ordering(kfp.RED_BLACK)
    kfp.set_pipeline(inflight)
    bad = np.zeros((2 * (J - 1), nt, nx))
    bad[1, 3, 5] = np.inf
    uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, 2, R, p=4.0, tol=1e-11, max_iter=300,
                              lambda_init=dev(bad))
    assert st.restarted
    ref = oracle.swr_solve(u0, f, T, nt, J, 2, R, p=4.0, tol=1e-11, max_iter=300, order=1)
    assert st.iters == ref.iters and rel(host(uT), ref.uT) <= 1e-10
    with pytest.raises(kfp.KfpError):
        kfp.swr_solve(dev(u0), dev(f), T, nt, J, 2, R, p=4.0, tol=1e-14, max_iter=2,
                      raise_noconv=True)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, J, 2, R, p=4.0, tol=1e-14, max_iter=2,
                                want_lambda=True)
    ref = oracle.swr_solve(u0, f, T, nt, J, 2, R, p=4.0, tol=1e-14, max_iter=2, order=1)
    assert st.iters == 2 and ref.status == 4
    assert rel(host(uT), ref.uT) <= 1e-12 and rel(host(lam), ref.lam) <= 1e-12


def test_windows_report_a_window_that_does_not_converge():
    nx, nv, nt, T = 48, 64, 30, 0.2
    u0, f = inputs.random_fields(4, nx, nv)
    uT, its, st = kfp.swr_solve_windows(dev(u0), dev(f), T, nt, 2, 2, R, p=4.0, tol=1e-15,
                                        max_iter=3, n_windows=3)
    assert its == [3, 3, 3] and st.iters == 9 and not st.residual < 1e-15
    ref, rit, rst = oracle.swr_solve_windows(u0, f, T, nt, 2, 2, R, p=4.0, tol=1e-15,
                                             max_iter=3, n_windows=3)
    assert rit == its and all(x == 4 for x in rst)
    assert rel(host(uT), ref) <= 1e-12


def test_red_black_rejects_the_one_step_kernel():
    nx, nv, nt, T = 32, 64, 10, 0.1
    u0, f = inputs.random_fields(3, nx, nv)
    kfp.set_ordering(kfp.RED_BLACK)
    kfp.set_config(4, 0, 0)
    with pytest.raises(kfp.KfpError):
        kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 2, R, p=4.0, tol=1e-10, max_iter=10)


# ------------------------------------------------- the paper's experiments --
def test_table1_trends_on_the_gpu():
    """Section 6.5, Table 1 at levels j = 0..2 through the library (two
    subdomains, T = 2, error equation, 1e-6).  Counts are parity unpinned
    (different discretisation and order); the trends the paper reports must
    hold: OSWR converges far faster than CSWR, whose mismatch after the cap
    grows under refinement; the two-sided variant degrades less under
    refinement than the one-sided one; without overlap OSWR still converges,
    with more iterations than with overlap.  Level 0 also matches the
    oracle's counts."""
    from paper_1306_4596_amd import experiments as ex

    res = {}
    for j in (0, 1, 2):
        nx, nv, nt, z, lam0 = ex._zero_problem(j)
        for key, tr, o, p, q, cap in (("C", D, 3, 0.0, None, 150), ("P", R, 3, ex.PSTAR, None, 400),
                                      ("PQ", R, 3, ex.P2, ex.Q2, 400), ("P0", R, 0, ex.PSTAR, None, 400)):
            _, _, st = kfp.swr_solve(z, z, ex.T_END, nt, 2, o, tr, p=p, q=q, tol=ex.TOL,
                                     max_iter=cap, lambda_init=lam0)
            res[key, j] = (st.iters, st.residual)
    for j in (0, 1, 2):
        assert res["C", j][1] > ex.TOL            # CSWR: not converged after 150
        assert res["P", j][1] < ex.TOL and res["P", j][0] < 75
        assert res["P0", j][1] < ex.TOL and res["P0", j][0] > res["P", j][0]
    assert res["C", 0][1] < res["C", 1][1] < res["C", 2][1]
    gp = res["P", 2][0] / res["P", 0][0]
    gpq = res["PQ", 2][0] / res["PQ", 0][0]
    assert gpq < gp
    nx, nv, nt = ex.grid(0)
    lam0 = inputs.random_traces(0, 2, nt, nx)
    zz = np.zeros((nv + 1, nx))
    ref = oracle.swr_solve(zz, zz, ex.T_END, nt, 2, 3, R, p=ex.PSTAR, tol=ex.TOL, max_iter=400,
                           lambda_init=lam0)
    assert res["P", 0][0] == ref.iters


# ------------------------------------------------------------ time windows --
WINDOW_CASES = [
    # nx, nv, nt, T, J, o, tr, p, q, windows, guess, ordering
    (48, 64, 37, 0.2, 2, 2, R, 4.0, None, 4, False, 0),
    (48, 64, 37, 0.2, 4, 2, R, 3.0, 1.5, 5, True, 0),
    (40, 64, 12, 0.1, 2, 4, D, 0.0, None, 12, True, 0),
    (64, 96, 30, 0.2, 3, 0, R, 5.0, None, 3, True, 1),
    (32, 32, 20, 0.1, 1, 0, D, 0.0, None, 2, False, 0),
]


@pytest.mark.parametrize("case", WINDOW_CASES)
def test_time_windows_match_oracle(case):
    nx, nv, nt, T, J, o, tr, p, q, W, guess, order = case
    print(f"windows case={case}", flush=True)
    u0, f = inputs.random_fields(90 + W, nx, nv)
    s = 1.0 + 0.3 * np.cos(np.arange(nt + 1))
    kfp.set_ordering(order)
    ref, rit, _ = oracle.swr_solve_windows(u0, f, T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                                           max_iter=400, n_windows=W, s=s, guess=guess)
    if order:  # the oracle in the same order
        start = u0
        rit = []
        for w in range(W):
            n0, n1 = w * nt // W, (w + 1) * nt // W
            lam0 = oracle.u0_guess(start, n1 - n0, J, o, tr, p, q) if guess and J > 1 else None
            r = oracle.swr_solve(start, f, (n1 - n0) * (T / nt), n1 - n0, J, o, tr, p=p, q=q,
                                 tol=1e-11, max_iter=400, lambda_init=lam0, s=s[n0:n1 + 1],
                                 order=1)
            rit.append(r.iters)
            start = r.uT
        ref = start
    uT, its, st = kfp.swr_solve_windows(dev(u0), dev(f), T, nt, J, o, tr, p=p, q=q, tol=1e-11,
                                        max_iter=400, n_windows=W, s=s, guess=guess)
    assert its == rit and st.iters == sum(rit)
    assert rel(host(uT), ref) <= 1e-10
    m = oracle.mono_solve(u0, f, T, nt, s)
    assert rel(host(uT), m) <= 1e-9


# ------------------------------------------------- overlapped iterations ----
PIPE_CASES = [
    # nx, nv, nt, T, J, o, tr, p, (waves, seg, steps[, groups]) or None
    (64, 64, 60, 0.3, 4, 2, R, 4.0, None),
    (64, 64, 200, 0.1, 2, 4, D, 0.0, None),
    (100, 96, 41, 0.2, 3, 3, R, 2.5, (4, 12, 4)),
    (70, 120, 30, 0.2, 8, 1, D, 0.0, (2, 12, 3)),
    (200, 128, 64, 0.25, 4, 5, R, 8.0, (4, 12, 8)),
    (64, 256, 40, 0.2, 2, 2, R, 4.0, (8, 17, 4, 2)),
]


@pytest.mark.parametrize("case", PIPE_CASES)
@pytest.mark.parametrize("inflight", [2, 3, 7])
def test_overlapped_iterations_equal_plain_iterations(case, inflight):
    """Iterations overlapped in time reproduce the plain iteration exactly:
    iterate, traces, count and residual history, bit for bit."""
    nx, nv, nt, T, J, o, tr, p, cfg = case
    print(f"pipeline case={case} inflight={inflight}", flush=True)
    if cfg:
        kfp.set_config(*cfg)
    u0, f = inputs.random_fields(21, nx, nv)
    runs = []
    for mode in (0, inflight):
        kfp.set_pipeline(mode)
        runs.append(kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-11, max_iter=400,
                                  want_lambda=True))
    (a, la, sa), (b, lb, sb) = runs
    assert sa.iters == sb.iters and sa.residual < 1e-11
    assert torch.equal(a, b) and torch.equal(la, lb)
    assert np.array_equal(sa.res_history, sb.res_history)
    # and the fixed-count form (stops at max_iter, not at the tolerance)
    kfp.set_pipeline(inflight)
    c, lc, sc = kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-300, max_iter=5,
                              want_lambda=True)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-300, max_iter=5)
    assert sc.iters == 5
    assert rel(host(c), ref.uT) <= 1e-12
    assert rel(host(lc), ref.lam) <= 1e-12
    assert np.allclose(sc.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)


def test_overlapped_iterations_with_guess_and_restart():
    nx, nv, nt, T = 64, 32, 40, 0.2
    u0, f = inputs.random_fields(2, nx, nv)
    kfp.set_pipeline(4)
    bad = np.zeros((6, nt, nx))
    bad[0, 3, 5] = np.nan
    uT, _, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=4.0, tol=1e-11, max_iter=300,
                              lambda_init=dev(bad))
    assert st.restarted
    ref = oracle.swr_solve(u0, f, T, nt, 4, 2, R, p=4.0, tol=1e-11, max_iter=300)
    assert st.iters == ref.iters
    assert rel(host(uT), ref.uT) <= 1e-10
    lam0 = inputs.random_traces(3, 4, nt, nx)
    ref = oracle.swr_solve(u0, f, T, nt, 4, 2, R, p=4.0, tol=1e-300, max_iter=4, lambda_init=lam0)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 4, 2, R, p=4.0, tol=1e-300, max_iter=4,
                                lambda_init=dev(lam0), want_lambda=True)
    assert not st.restarted and st.iters == 4
    assert rel(host(lam), ref.lam) <= 1e-12


# ------------------------------------------------------------------ batch --
@pytest.mark.parametrize("cfg", [(16, 32, 0), (16, 12, 6), (8, 24, 1), (8, 17, 4, 2)])
def test_batch_matches_single_solves(cfg):
    specs = [
        (64, 64, 40, 0.2, 2, 2, R, 4.0),
        (128, 32, 40, 0.1, 4, 2, R, 2.0),
        (96, 128, 40, 0.3, 8, 2, D, 0.0),
        (64, 256, 40, 0.2, 2, 3, R, 8.0),
        (256, 64, 40, 0.15, 1, 0, R, 1.0),
    ]
    insts, refs = [], []
    kfp.set_config(*cfg)  # one configuration for the batch and the singles
    for i, (nx, nv, nt, T, J, o, tr, p) in enumerate(specs):
        u0, f = inputs.random_fields(100 + i, nx, nv)
        insts.append(dict(u0=dev(u0), f=dev(f), T=T, nt=nt, J=J, overlap=o, tr=tr, p=p,
                          want_lambda=True))
        refs.append(kfp.swr_solve(dev(u0), dev(f), T, nt, J, o, tr, p=p, tol=1e-11, max_iter=400,
                                  want_lambda=True))
    out, rc = kfp.swr_batch(insts, tol=1e-11, max_iter=400, history=True)
    assert rc == 0
    kfp.set_config(0)
    for (uT, lam, st), (ruT, rlam, rst) in zip(out, refs):
        assert st.iters == rst.iters
        assert torch.equal(uT, ruT)
        if lam is not None:
            assert torch.equal(lam, rlam)
    # and against the oracle
    for (nx, nv, nt, T, J, o, tr, p), (uT, _, st), i in zip(specs, out, range(len(specs))):
        u0, f = inputs.random_fields(100 + i, nx, nv)
        ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-11, max_iter=400)
        assert st.iters == ref.iters
        assert rel(host(uT), ref.uT) <= 1e-10


# ------------------------------------------------------ full-size checks ----
def test_many_items_register_limited_build():
    """8 wavefronts x 17 rows with at least two work items per compute unit
    runs the build limited to 128 registers: 3072 x 1024, J = 8 at 8 steps
    per launch (512 items), two iterations against the oracle."""
    nx, nv, nt, T = 3072, 1024, 24, 0.005
    u0, f = inputs.random_fields(8, nx, nv)
    print("many items oracle ...", flush=True)
    ref = oracle.swr_solve(u0, f, T, nt, 8, 2, R, p=8.0, tol=1e-300, max_iter=2)
    kfp.set_config(8, 17, 8)
    kfp.set_pipeline(0)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 8, 2, R, p=8.0, tol=1e-300, max_iter=2,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12


def test_tall_subdomains_full_size_fixed_iterations():
    """1024 x 1024 with J = 2 (514-row subdomains, the built-in lane-group
    march): two iterations against the oracle."""
    nx = nv = 1024
    nt, T = 40, 0.01
    u0, f = inputs.random_fields(5, nx, nv)
    print("tall subdomains oracle ...", flush=True)
    ref = oracle.swr_solve(u0, f, T, nt, 2, 2, R, p=4.0, tol=1e-300, max_iter=2)
    assert kfp.get_launch(nx, nv, nt, T, 2, 2, R)[3] >= 2
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 2, 2, R, p=4.0, tol=1e-300, max_iter=2,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12


def test_cfg1_shape_fixed_iterations_short_window():
    """The 1024 x 1024, J = 8, overlap 2, Robin shape of the benchmark, with
    the same dt but a 200-step window: two iterations against the oracle."""
    nx = nv = 1024
    nt, T = 200, 0.05
    u0, f = inputs.random_fields(0, nx, nv)
    print("cfg1 shape oracle ...", flush=True)
    ref = oracle.swr_solve(u0, f, T, nt, 8, 2, R, p=4.0, tol=1e-300, max_iter=2)
    uT, lam, st = kfp.swr_solve(dev(u0), dev(f), T, nt, 8, 2, R, p=4.0, tol=1e-300, max_iter=2,
                                want_lambda=True)
    assert rel(host(uT), ref.uT) <= 1e-12
    assert rel(host(lam), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9)


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48])
def test_bw_probe_copies(nbytes):
    """The bandwidth probe is a plain copy: bit-exact, whole and ragged
    workgroups, and nothing written past the requested bytes."""
    n = nbytes // 8
    src = torch.arange(n + 4, dtype=torch.float64, device="cuda") * 0.5 + 1.0
    dst = torch.full((n + 4,), -7.0, dtype=torch.float64, device="cuda")
    binding._check(binding.load_library().kfp_bw_probe(ctypes.c_void_p(src.data_ptr()),
                                                       ctypes.c_void_p(dst.data_ptr()),
                                                       int(nbytes), None))
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src[:n])
    assert bool((dst[n:] == -7.0).all())


@pytest.mark.parametrize("waves,rpw", [(8, 17), (8, 9), (4, 1)])
def test_tile_probe_writes_u_plus_half_f(waves, rpw):
    """The tile-shaped streaming probe: V = U + F/2 (one FMA, exact here for
    these binary fractions), a ragged last tile and row block, nothing
    written past the last row."""
    rows, nx = 300, 200
    U = torch.arange(rows * nx, dtype=torch.float64, device="cuda").reshape(rows, nx) * 0.25
    F = torch.full((rows, nx), 3.0, dtype=torch.float64, device="cuda")
    Vb = torch.full((rows + 1, nx), -7.0, dtype=torch.float64, device="cuda")
    V = Vb[:rows]
    assert kfp.tile_probe(U, F, V, waves, rpw) == 24 * rows * nx
    torch.cuda.synchronize()
    assert torch.equal(V, U + 1.5)
    assert bool((Vb[rows] == -7.0).all())

"""GPU tests of the x-Fourier trace helpers (kfp_trace_modes,
kfp_trace_synth) against their plain definitions, the claim they rest on
(fields of the x frequencies 1..4 give traces of exactly those frequencies),
and the coarse-grid learned guess built on them."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1306_4596_amd as kfp  # noqa: E402
from paper_1306_4596_amd import inputs, learned  # noqa: E402

pytestmark = pytest.mark.gpu
MODES = inputs.X_FREQS


def ref_modes(lam, modes):
    nx = lam.shape[-1]
    i = np.arange(nx)
    out = []
    for m in modes:
        out.append((2.0 / nx) * (lam * np.cos(2 * np.pi * m * i / nx)).sum(-1))
        out.append((2.0 / nx) * (lam * np.sin(2 * np.pi * m * i / nx)).sum(-1))
    return np.stack(out, -1)


def ref_synth(coef, modes, nt, nx):
    P, ntc, _ = coef.shape
    i = np.arange(nx)
    out = np.empty((P, nt, nx))
    for n in range(nt):
        sc = (n + 1) * ntc / nt - 1.0
        if sc <= 0:
            k0 = k1 = 0
            w = 0.0
        elif sc >= ntc - 1:
            k0 = k1 = ntc - 1
            w = 0.0
        else:
            k0 = int(math.floor(sc))
            k1 = k0 + 1
            w = sc - k0
        c = coef[:, k0] + w * (coef[:, k1] - coef[:, k0])
        v = np.zeros((P, nx))
        for k, m in enumerate(modes):
            v += c[:, 2 * k, None] * np.cos(2 * np.pi * m * i / nx)[None, :]
            v += c[:, 2 * k + 1, None] * np.sin(2 * np.pi * m * i / nx)[None, :]
        out[:, n] = v
    return out


@pytest.mark.parametrize("rows,nx,modes", [(37, 64, MODES), (5, 10, (1, 4)), (300, 512, (3,)),
                                           (3, 4096, (1, 2, 3, 4, 5, 6, 7, 8))])
def test_trace_modes_matches_definition(rows, nx, modes):
    print(f"trace_modes rows={rows} nx={nx} modes={modes}", flush=True)
    lam = np.random.default_rng(rows).standard_normal((rows, nx))
    got = kfp.trace_modes(torch.from_numpy(lam).cuda(), modes).cpu().numpy()
    ref = ref_modes(lam, modes)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("P,ntc,nt,nx,modes", [(3, 5, 11, 48, MODES), (2, 8, 8, 16, (1, 7)),
                                               (4, 16, 5, 33, (2, 5)), (1, 1, 3, 300, MODES)])
def test_trace_synth_matches_definition(P, ntc, nt, nx, modes):
    print(f"trace_synth P={P} ntc={ntc} nt={nt} nx={nx}", flush=True)
    coef = np.random.default_rng(P * 100 + ntc).standard_normal((P, ntc, 2 * len(modes)))
    got = kfp.trace_synth(torch.from_numpy(coef).cuda(), modes, nt, nx).cpu().numpy()
    ref = ref_synth(coef, modes, nt, nx)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("J,o", [(4, 2), (8, 1)])
def test_solver_traces_hold_only_the_field_frequencies(J, o):
    """Every operator is circulant in x, so traces of fields with the x
    frequencies 1..4 have exactly those: projecting the converged traces
    and synthesising them on the same grid gives them back."""
    nx, nv, nt = 64, 64, 128
    print(f"traces of the field frequencies J={J} o={o}", flush=True)
    u0, f = inputs.random_fields(3, nx, nv)
    U0, F = torch.from_numpy(u0).cuda(), torch.from_numpy(f).cuda()
    _, lam, st = kfp.swr_solve(U0, F, 0.5, nt, J, o, kfp.ROBIN, p=4.0, tol=1e-10, max_iter=500,
                               want_lambda=True)
    c = kfp.trace_modes(lam, MODES)
    back = kfp.trace_synth(c, MODES, nt, nx)
    scale = float(lam.abs().max())
    assert scale > 0
    assert float((back - lam).abs().max()) <= 1e-12 * scale


def test_coarse_learned_guess_shortens_the_fine_solve():
    """A modal guess trained on coarse solves (same J, overlap, T and p)
    starts the fine solve of a held-out seed closer to its converged traces
    than zero traces do, and the solve needs fewer iterations; the solution
    is the same."""
    coarse = learned.Shape(32, 32, 64, 0.5, 4, 2, kfp.ROBIN, 4.0)
    fine = learned.Shape(128, 128, 256, 0.5, 4, 2, kfp.ROBIN, 4.0)
    print("coarse learned guess: training", flush=True)
    g, t_gen, t_train, cit = learned.train_modal_guess(coarse, range(1, 193), epochs=400)
    u0, f = inputs.random_fields(0, fine.nx, fine.nv)
    U0, F = torch.from_numpy(u0).cuda(), torch.from_numpy(f).cuda()
    kw = dict(p=fine.p, tol=1e-10, max_iter=500)
    u_zero, lam_star, st_zero = kfp.swr_solve(U0, F, fine.T, fine.nt, fine.J, fine.overlap,
                                              fine.tr, want_lambda=True, **kw)
    lam0 = g.predict(inputs.coefficients(0), fine.nt, fine.nx)[0].contiguous()
    gerr = float((lam0 - lam_star).abs().max() / lam_star.abs().max())
    u_l, _, st_l = kfp.swr_solve(U0, F, fine.T, fine.nt, fine.J, fine.overlap, fine.tr,
                                 lambda_init=lam0, **kw)
    print(f"guess error {gerr:.3e}; iterations zero {st_zero.iters} learned {st_l.iters}; "
          f"coarse iterations {cit:.1f}", flush=True)
    assert gerr < 0.25
    assert st_l.iters < st_zero.iters
    assert float((u_l - u_zero).norm() / u_zero.norm()) <= 1e-10


@pytest.mark.parametrize("W,order", [(3, kfp.PARALLEL), (4, kfp.RED_BLACK)])
def test_windows_from_whole_interval_traces(W, order):
    """kfp_swr_solve_windows_init: each window starts from its levels of
    traces given for the whole interval.  From zero traces it is the
    windowed solve from zero bit for bit; from the converged traces of the
    single-window solve every window starts at its own solution (a few
    iterations); both compose to the monodomain solution of the oracle."""
    nx, nv, nt, T, J, o, p = 64, 96, 120, 0.3, 4, 2, 4.0
    print(f"windows from whole-interval traces W={W} order={order}", flush=True)
    u0, f = inputs.random_fields(11, nx, nv)
    U0, F = torch.from_numpy(u0).cuda(), torch.from_numpy(f).cuda()
    try:
        kfp.set_ordering(order)
        kw = dict(p=p, tol=1e-11, max_iter=400, n_windows=W)
        u_z, it_z, _ = kfp.swr_solve_windows(U0, F, T, nt, J, o, kfp.ROBIN, **kw)
        zeros = torch.zeros((2 * (J - 1), nt, nx), dtype=torch.float64, device="cuda")
        u_0, it_0, _ = kfp.swr_solve_windows(U0, F, T, nt, J, o, kfp.ROBIN, lambda_init=zeros, **kw)
        assert it_0 == it_z and torch.equal(u_0, u_z)
        _, lam_star, _ = kfp.swr_solve(U0, F, T, nt, J, o, kfp.ROBIN, p=p, tol=1e-13,
                                       max_iter=600, want_lambda=True)
        u_s, it_s, _ = kfp.swr_solve_windows(U0, F, T, nt, J, o, kfp.ROBIN, lambda_init=lam_star,
                                             **kw)
        assert max(it_s) <= 3 < min(it_z)
    finally:
        kfp.set_ordering(kfp.PARALLEL)
    m = oracle.mono_solve(u0, f, T, nt)
    for u in (u_z, u_s):
        assert np.linalg.norm(u.cpu().numpy() - m) / np.linalg.norm(m) <= 1e-9

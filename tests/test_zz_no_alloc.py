"""The entry point that allocates nothing (kfp_mono_solve_static) against the
allocating one (kfp_mono_solve) and the CPU oracle, through the C ABI.

Both entry points run the same kernels on the same tables, so their outputs
agree bit for bit; against the oracle the monodomain march is held to
relative L2 <= 1e-12 (the same arithmetic up to the rounding order of the
elimination).  Two calls in a row share the static workspace, the second on
a smaller grid, so a stale table or state left by the first call would show.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1306_4596_amd as kfp  # noqa: E402
from paper_1306_4596_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("scheme", ["fd", "fem"])
def test_static_mono_matches_allocating_entry_point(scheme):
    kfp.set_scheme(kfp.FEM if scheme == "fem" else kfp.FD)
    try:
        # the second call is smaller: fewer rows, columns and steps
        for seed, (nx, nv, nt, T) in enumerate([(256, 512, 300, 0.2), (100, 40, 37, 0.2)]):
            print(f"no-alloc mono {scheme} nx={nx} nv={nv} nt={nt}", flush=True)
            u0, f = inputs.random_fields(seed + 7, nx, nv)
            s = 1.0 + 0.5 * np.sin(np.arange(nt + 1))
            a = kfp.mono_solve_static(dev(u0), dev(f), T, nt, s=s)
            torch.cuda.synchronize()
            b = kfp.mono_solve(dev(u0), dev(f), T, nt, s=s)
            torch.cuda.synchronize()
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.array_equal(a, b)
            ref = oracle.mono_solve(u0, f, T, nt, s,
                                    scheme=oracle.FEM if scheme == "fem" else oracle.FD)
            assert rel(a, ref) <= 1e-12
    finally:
        kfp.set_scheme(kfp.FD)


def test_static_mono_rejects_grids_beyond_the_workspace():
    nx, nv, nt, T = 4096, 4096, 100, 0.01
    u0 = torch.zeros((nv + 1, nx), dtype=torch.float64, device="cuda")
    with pytest.raises(kfp.KfpError, match="static workspace"):
        kfp.mono_solve_static(u0, u0, T, nt)

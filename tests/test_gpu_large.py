"""GPU parity at the largest workload's shape: 4096 x 4096, J = 32, overlap 2,
Robin p = 8, in the launch configuration the library chooses for it (8
wavefronts x 17 rows and the 128-register build, more than two work items
per compute unit: finite differences on the multi-tile kernel with one tile
at 12 steps per launch, finite elements on the general march kernel at 8).  The window is cut to 16 steps
(T = 16 / 4096, the same Courant numbers as a CFL-limited step) so that the
oracle finishes in seconds; two iterations are compared element by element
(traces and glued output), in both discretisations."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1306_4596_amd as kfp  # noqa: E402
from paper_1306_4596_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def _reset():
    kfp.set_config(0)
    kfp.set_pipeline(-1)
    kfp.set_ordering(kfp.PARALLEL)
    kfp.set_scheme(kfp.FD)
    yield
    kfp.set_scheme(kfp.FD)
    kfp.release_workspace()


@pytest.mark.parametrize("scheme", [oracle.FD, oracle.FEM])
def test_largest_shape_two_iterations(scheme):
    nx = nv = 4096
    nt = 16
    T = nt / 4096.0
    J, o, p = 32, 2, 8.0
    u0, f = inputs.random_fields(0, nx, nv)
    print(f"4096^2 J=32 scheme={scheme}: oracle ...", flush=True)
    ref = oracle.swr_solve(u0, f, T, nt, J, o, oracle.ROBIN, p=p, tol=1e-300, max_iter=2,
                           scheme=scheme)
    kfp.set_scheme(kfp.FEM if scheme == oracle.FEM else kfp.FD)
    cfg = kfp.get_launch_tiles(nx, nv, nt, T, J, o, kfp.ROBIN)
    if scheme == oracle.FEM:
        assert cfg == (8, 17, 8, 1, 0), cfg
    else:  # the multi-tile kernel, one tile, 12 steps per launch (the last one 4)
        assert cfg == (8, 17, 12, 1, 1), cfg
    print(f"4096^2 J=32 scheme={scheme}: GPU, launch {cfg}", flush=True)
    uT, lam, st = kfp.swr_solve(torch.from_numpy(u0).cuda(), torch.from_numpy(f).cuda(), T, nt,
                                J, o, kfp.ROBIN, p=p, tol=1e-300, max_iter=2, want_lambda=True)
    assert st.iters == 2
    assert rel(uT.cpu().numpy(), ref.uT) <= 1e-12
    assert rel(lam.cpu().numpy(), ref.lam) <= 1e-12
    assert np.allclose(st.res_history, ref.res_hist, rtol=1e-9, atol=1e-14)

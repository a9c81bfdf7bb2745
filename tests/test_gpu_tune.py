"""The launch-configuration autotuner (kfp_tune): it times the compiled
configurations that hold a shape, caches the fastest per shape and
discretisation, and later solves of that shape use it."""
import json
import os

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
    yield
    kfp.set_scheme(kfp.FD)


def test_autotuner_choice_is_cached_and_used(tmp_path, monkeypatch):
    cache = tmp_path / "a" / "b" / "tune.json"  # folders created by the library
    monkeypatch.setenv("KFP_TUNE_CACHE", str(cache))
    # a shape no other test uses (the choice stays in the process's table)
    nx, nv, nt, T, J, o, p = 36, 48, 24, 0.2, 2, 2, 4.0
    u0, f = inputs.random_fields(36, nx, nv)
    for scheme in (oracle.FD, oracle.FEM):
        print(f"tune scheme={scheme}", flush=True)
        kfp.set_scheme(kfp.FEM if scheme == oracle.FEM else kfp.FD)
        w, seg, k = kfp.tune(nx, nv, nt, T, J, o, kfp.ROBIN, p=p)
        assert w in (1, 2, 4, 8, 16) and seg >= 0 and k >= 0
        if scheme == oracle.FEM:
            assert k >= 1  # the finite-element scheme runs on the march kernel only
        assert kfp.get_launch(nx, nv, nt, T, J, o, kfp.ROBIN)[:3] == (w, seg, k)
        ref = oracle.swr_solve(u0, f, T, nt, J, o, oracle.ROBIN, p=p, tol=1e-11, max_iter=300,
                               scheme=scheme)
        uT, _, st = kfp.swr_solve(torch.from_numpy(u0).cuda(), torch.from_numpy(f).cuda(), T,
                                  nt, J, o, kfp.ROBIN, p=p, tol=1e-11, max_iter=300)
        assert st.iters == ref.iters
        assert rel(uT.cpu().numpy(), ref.uT) <= 1e-10
    assert os.path.exists(cache)
    keys = list(json.load(open(cache)))
    assert any(key.endswith("/fem") and "/nx36/" in key for key in keys), keys
    assert any(not key.endswith("/fem") and "/nx36/" in key for key in keys), keys


def test_tuned_one_step_choice_is_passed_over_in_red_black_order(tmp_path, monkeypatch):
    """A cached one-step configuration (steps = 0) of a shape serves the
    parallel order; a red-black solve of the same shape, which needs a march
    configuration, falls back to the built-in march choice and still
    matches the oracle."""
    nx, nv, nt, T, J, o, p = 40, 64, 30, 0.2, 2, 2, 4.0
    # Robin, J = 2, overlap 2: both subdomains hold 33 unknown rows
    key = f"gfx950/nx{nx}/nmax33/J{J}/tr1"
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({key: [4, 16, 0, 1]}))
    monkeypatch.setenv("KFP_TUNE_CACHE", str(cache))
    kfp.reload_tune_cache()
    try:
        assert kfp.get_launch(nx, nv, nt, T, J, o, kfp.ROBIN) == (4, 16, 0, 1)
        kfp.set_ordering(kfp.RED_BLACK)
        w, seg, k, g = kfp.get_launch(nx, nv, nt, T, J, o, kfp.ROBIN)
        assert k >= 1, (w, seg, k, g)
        u0, f = inputs.random_fields(40, nx, nv)
        print("red-black solve with a cached one-step choice", flush=True)
        uT, _, st = kfp.swr_solve(torch.from_numpy(u0).cuda(), torch.from_numpy(f).cuda(), T,
                                  nt, J, o, kfp.ROBIN, p=p, tol=1e-11, max_iter=300)
        ref = oracle.swr_solve(u0, f, T, nt, J, o, oracle.ROBIN, p=p, tol=1e-11, max_iter=300,
                               order=1)
        assert st.iters == ref.iters
        assert rel(uT.cpu().numpy(), ref.uT) <= 1e-10
    finally:
        kfp.set_ordering(kfp.PARALLEL)
        monkeypatch.undo()
        kfp.reload_tune_cache()


def test_batch_tuner_classes_are_used_by_the_batch(tmp_path, monkeypatch):
    """kfp_tune_batch times the configurations of every subdomain height of a
    batch and caches the winners; kfp_swr_batch then runs each launch class
    in its tuned configuration, with results bit for bit those of single
    solves in that configuration and matching the oracle."""
    cache = tmp_path / "batch_tune.json"
    monkeypatch.setenv("KFP_TUNE_CACHE", str(cache))
    kfp.reload_tune_cache()
    specs = [  # nx, nv, nt, T, J, o, tr, p: four subdomain heights
        (64, 64, 40, 0.2, 2, 2, kfp.ROBIN, 4.0),
        (128, 32, 40, 0.1, 4, 2, kfp.ROBIN, 2.0),
        (96, 128, 40, 0.3, 8, 2, kfp.DIRICHLET, 0.0),
        (200, 128, 40, 0.2, 4, 3, kfp.ROBIN, 8.0),
        (80, 64, 40, 0.2, 2, 2, kfp.ROBIN, 3.0),
    ]
    insts = []
    for i, (nx, nv, nt, T, J, o, tr, p) in enumerate(specs):
        u0, f = inputs.random_fields(500 + i, nx, nv)
        insts.append(dict(u0=torch.from_numpy(u0).cuda(), f=torch.from_numpy(f).cuda(), T=T,
                          nt=nt, J=J, overlap=o, tr=tr, p=p, want_lambda=True))
    print("tuning the batch", flush=True)
    assert kfp.tune_batch(insts, iters=2) == 4
    kfp.reload_tune_cache()
    table = json.load(open(cache))
    batch_keys = [k for k in table if "/batch/nmax" in k]
    assert len(batch_keys) == 4, table
    out, rc = kfp.swr_batch(insts, tol=1e-11, max_iter=400)
    assert rc == 0
    for i, ((nx, nv, nt, T, J, o, tr, p), (uT, lam, st)) in enumerate(zip(specs, out)):
        w, seg, k, g, tl = kfp.get_batch_launch(insts[i])
        # the class configuration is one of the tuned entries
        assert [w, seg, k, g, tl] in [table[key] for key in batch_keys]
        kfp.set_config(w, seg, k, groups=g, tiles=tl)
        ruT, rlam, rst = kfp.swr_solve(insts[i]["u0"], insts[i]["f"], T, nt, J, o, tr, p=p,
                                       tol=1e-11, max_iter=400, want_lambda=True)
        kfp.set_config(0)
        assert st.iters == rst.iters
        assert torch.equal(uT, ruT)
        u0, f = inputs.random_fields(500 + i, nx, nv)
        ref = oracle.swr_solve(u0, f, T, nt, J, o, tr, p=p, tol=1e-11, max_iter=400)
        assert st.iters == ref.iters
        assert rel(uT.cpu().numpy(), ref.uT) <= 1e-10
    kfp.reload_tune_cache()

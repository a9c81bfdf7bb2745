"""The learned initial traces, end to end on a reduced shape: solves of the
method generate the training set, the library's kernels train the network,
and on held-out seeds the learned guess reaches the same tolerance and the
same solution in fewer SWR iterations than the zero guess."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1306_4596_amd as kfp  # noqa: E402
from paper_1306_4596_amd import learned  # noqa: E402

pytestmark = pytest.mark.gpu


def test_learned_guess_saves_iterations():
    shape = learned.Shape(64, 64, 64, 0.25, 4, 2, kfp.ROBIN, 4.0)
    print("generating", flush=True)
    X, Y, iters = learned.generate(shape, range(512), batch=128, tol=1e-10)
    assert np.all(iters > 0)
    guess = learned.LearnedGuess(shape, hidden=256, depth=3, seed=1)
    print("training", flush=True)
    hist = guess.fit(X, Y, epochs=300, batch=32, lr=2e-3, lr_min=1e-6)
    print("loss", hist[0], hist[-1], flush=True)
    assert hist[-1] < 0.01 * hist[0]
    ev = learned.evaluate(shape, range(10000, 10012), guess, tol=1e-10)
    z = np.array([r["iters"] for r in ev["zero"]])
    l_ = np.array([r["iters"] for r in ev["learned"]])
    print("zero", z, "learned", l_, "u0", [r["iters"] for r in ev["u0"]], flush=True)
    assert all(r["residual"] < 1e-10 for r in ev["learned"])
    # both runs stop at an absolute residual of 1e-10: the same discrete solution
    assert max(r["rel_l2_vs_zero_guess"] for r in ev["learned"]) < 1e-8
    assert l_.mean() < z.mean() - 2
    assert not any(r["restarted"] for r in ev["learned"])

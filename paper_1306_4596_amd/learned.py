"""Learned initial interface traces for SWR.

A network maps the 64 coefficients of the seeded fields (u0, f) to the
converged interface traces of one problem shape.  It is trained on solves the
SWR path itself generates (kfp_swr_batch), with the library's own forward,
backward and Adam kernels.  At solve time its prediction is the initial guess
lambda^0; the SWR iteration still runs to the same tolerance, so it is both
the fallback and the judge of the network's error.

    python -m paper_1306_4596_amd.learned --train 20000 --eval 2000 --out results.json
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import asdict, dataclass

import numpy as np

from . import binding as kb
from . import inputs


@dataclass
class Shape:
    nx: int
    nv: int
    nt: int
    T: float
    J: int
    overlap: int
    tr: int
    p: float

    @property
    def n_out(self):
        return 2 * (self.J - 1) * self.nt * self.nx


# 256 x 256, Nt = 512, J = 4, overlap 2, Robin p = 4
SHAPE_256 = Shape(256, 256, 512, 0.5, 4, 2, kb.ROBIN, 4.0)


def coef_matrix(seeds):
    return np.stack([inputs.coefficients(int(s)) for s in seeds]).astype(np.float64)


class FieldMaker:
    """Fields of many seeds at once: (u0, f) = coefficients x mode basis."""

    def __init__(self, shape: Shape):
        Bf, Bu = inputs.mode_basis(shape.nx, shape.nv)
        self.n = (shape.nv + 1) * shape.nx
        self.Bf = Bf.reshape(Bf.shape[0], -1)
        self.Bu = Bu.reshape(Bu.shape[0], -1)
        self.shape = shape

    def make(self, C):
        nm = inputs.N_MODES
        f = C[:, : 2 * nm] @ self.Bf
        u0 = C[:, 2 * nm:] @ self.Bu
        s = self.shape
        f = f.reshape(-1, s.nv + 1, s.nx)
        u0 = u0.reshape(-1, s.nv + 1, s.nx)
        f[:, 0] = 0.0
        f[:, -1] = 0.0
        return np.ascontiguousarray(u0), np.ascontiguousarray(f)


def generate(shape: Shape, seeds, batch=128, tol=1e-10, max_iter=500, log=None):
    """Converged traces of every seed (FP32, [N][n_out]) and their coefficients
    ([N][64] FP32), both on the GPU; plus the iteration counts."""
    import torch

    seeds = list(seeds)
    N = len(seeds)
    C = coef_matrix(seeds)
    X = torch.from_numpy(C.astype(np.float32)).cuda()
    Y = torch.empty((N, shape.n_out), dtype=torch.float32, device="cuda")
    iters = np.zeros(N, dtype=np.int32)
    fm = FieldMaker(shape)
    t0 = time.time()
    for b0 in range(0, N, batch):
        b1 = min(N, b0 + batch)
        u0s, fs = fm.make(C[b0:b1])
        U0 = torch.from_numpy(u0s).cuda()
        F = torch.from_numpy(fs).cuda()
        insts = [dict(u0=U0[i], f=F[i], T=shape.T, nt=shape.nt, J=shape.J, overlap=shape.overlap,
                      tr=shape.tr, p=shape.p, want_lambda=True) for i in range(b1 - b0)]
        res, rc = kb.swr_batch(insts, tol=tol, max_iter=max_iter)
        if rc != 0:
            raise RuntimeError("training solve did not converge")
        for i, (_, lam, st) in enumerate(res):
            kb.cast_f64_f32(lam.reshape(-1), Y[b0 + i])
            iters[b0 + i] = st.iters
        if log:
            log(f"generated {b1}/{N} traces ({time.time() - t0:.1f} s, "
                f"mean iterations {iters[:b1].mean():.1f})")
    torch.cuda.synchronize()
    return X, Y, iters


class LearnedGuess:
    """Network + per-output standardisation of one problem shape."""

    def __init__(self, shape: Shape, hidden=512, depth=3, seed=0, net=None):
        self.shape = shape
        self.net = net if net is not None else kb.MLP(inputs.N_COEF, hidden, depth, shape.n_out,
                                                      seed=seed)
        self.mean = None
        self.std = None

    def fit(self, X, Y, epochs=30, batch=256, lr=1e-3, lr_min=1e-5, log=None, seed=0):
        """Standardises Y in place (per output) and trains with Adam on a
        cosine learning-rate schedule.  Returns the epoch losses."""
        import torch

        self.mean, self.std = kb.column_stats(Y, floor=1e-6)
        kb.standardize(Y, self.mean, self.std)
        N = X.shape[0]
        nb = max(1, N // batch)
        steps = epochs * nb
        rng = np.random.default_rng(seed)
        hist = []
        k = 0
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(N)).cuda()
            tot = 0.0
            for b in range(nb):
                idx = perm[b * batch:(b + 1) * batch]
                xb = X.index_select(0, idx).contiguous()
                yb = Y.index_select(0, idx).contiguous()
                cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * k / max(1, steps - 1)))
                tot += self.net.train_step(xb, yb, cur)
                k += 1
            hist.append(tot / nb)
            if log:
                log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e}")
        return hist

    def predict(self, coef):
        """Initial traces lambda^0 (FP64 [B][2(J-1)][nt][nx]) for coefficient rows."""
        import torch

        X = torch.as_tensor(np.asarray(coef, dtype=np.float32)).reshape(-1, inputs.N_COEF).cuda()
        Yp = self.net.forward(X)
        lam = kb.destandardize(Yp, self.mean, self.std)
        s = self.shape
        return lam.reshape(-1, 2 * (s.J - 1), s.nt, s.nx)

    def save(self, prefix):
        import torch

        self.net.save(prefix + ".net")
        torch.save({"mean": self.mean.cpu(), "std": self.std.cpu(), "shape": asdict(self.shape)},
                   prefix + ".std.pt")

    @classmethod
    def load(cls, prefix):
        import torch

        d = torch.load(prefix + ".std.pt", weights_only=True)
        g = cls(Shape(**d["shape"]), net=kb.MLP.load(prefix + ".net"))
        g.mean = d["mean"].cuda()
        g.std = d["std"].cuda()
        return g


def evaluate(shape: Shape, seeds, guess: LearnedGuess | None, tol=1e-10, max_iter=500, log=None):
    """Iterations and wall time to tolerance for zero, u0-extension and
    learned initial traces on each seed (single solves, synchronised)."""
    import torch

    fm = FieldMaker(shape)
    out = {"zero": [], "u0": [], "learned": []}
    C = coef_matrix(seeds)
    for i, s in enumerate(seeds):
        u0s, fs = fm.make(C[i:i + 1])
        U0 = torch.from_numpy(u0s[0]).cuda()
        F = torch.from_numpy(fs[0]).cuda()
        runs = [("zero", None), ("u0", "u0")]
        if guess is not None:
            runs.append(("learned", "learned"))
        ref = None
        for name, kind in runs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam0 = None
            if kind == "u0":
                lam0 = kb.u0_guess(U0, shape.nt, shape.J, shape.overlap, shape.tr, shape.p)
            elif kind == "learned":
                lam0 = guess.predict(C[i])[0].contiguous()
            uT, _, st = kb.swr_solve(U0, F, shape.T, shape.nt, shape.J, shape.overlap, shape.tr,
                                     p=shape.p, tol=tol, max_iter=max_iter, lambda_init=lam0,
                                     history=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if ref is None:
                ref = uT
                err = 0.0
            else:
                err = float((uT - ref).norm() / ref.norm())
            out[name].append({"seed": int(s), "iters": st.iters, "seconds": dt,
                              "residual": st.residual, "rel_l2_vs_zero_guess": err,
                              "restarted": st.restarted})
        if log and (i + 1) % max(1, len(seeds) // 10) == 0:
            log(f"evaluated {i + 1}/{len(seeds)}")
    return out


def summarize(ev):
    res = {}
    for k, v in ev.items():
        if not v:
            continue
        it = np.array([r["iters"] for r in v], dtype=np.float64)
        sec = np.array([r["seconds"] for r in v])
        res[k] = {"n": len(v), "iters_mean": float(it.mean()), "iters_median": float(np.median(it)),
                  "iters_p90": float(np.percentile(it, 90)), "seconds_mean": float(sec.mean()),
                  "seconds_median": float(np.median(sec)),
                  "seconds_p90": float(np.percentile(sec, 90)),
                  "max_rel_l2_vs_zero_guess": float(max(r["rel_l2_vs_zero_guess"] for r in v))}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--eval", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--hidden", type=int, default=512)
    ap.add_argument("--out", default="learned_results.json")
    ap.add_argument("--save", default=None)
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    shape = SHAPE_256
    t0 = time.time()
    X, Y, iters = generate(shape, range(args.train), log=log)
    t_gen = time.time() - t0
    guess = LearnedGuess(shape, hidden=args.hidden)
    t0 = time.time()
    hist = guess.fit(X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    t_train = time.time() - t0
    del X, Y
    if args.save:
        guess.save(args.save)
    ev = evaluate(shape, range(20000, 20000 + args.eval), guess, log=log)
    res = {"shape": asdict(shape), "train_seeds": args.train, "eval_seeds": args.eval,
           "epochs": args.epochs, "generate_seconds": t_gen, "train_seconds": t_train,
           "train_iters_mean": float(iters.mean()), "loss_history": hist,
           "summary": summarize(ev)}
    with open(args.out, "w") as fp:
        json.dump(res, fp, indent=1)
    log(json.dumps(res["summary"]))


if __name__ == "__main__":
    main()

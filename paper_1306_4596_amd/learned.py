"""Learned initial interface traces for SWR.

A network maps the 64 coefficients of the seeded fields (u0, f) to the
converged interface traces of one problem shape.  It is trained on solves the
SWR path itself generates (kfp_swr_batch), with the library's own forward,
backward and Adam kernels.  At solve time its prediction is the initial guess
lambda^0; the SWR iteration still runs to the same tolerance, so it is both
the fallback and the measure of the network's error.

The map from coefficients to converged traces is linear (the equation and
the discretisation are linear, and the fields are linear in the
coefficients), so by default the output layer also reads the input: the GELU
trunk plus a linear map of the coefficients, whose accuracy is then bounded
by the BF16 rounding of weights and inputs rather than by how well GELU units
imitate a linear function away from the training data.

By default the network learns the correction to the u0-extension guess
(Q(u0) at every time level): lambda^0 = Q(u0) + net(coefficients).  The
correction is a small fraction of the traces, so the same relative error of a
BF16 network leaves a much smaller absolute error in lambda^0.  base="zero"
learns the traces themselves.

    python -m paper_1306_4596_amd.learned --train 20000 --eval 2000 --out results.json

`--scheme fem` does the same with the paper's finite-element discretisation
(training solves, targets and evaluation all in that scheme).
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
# 4096 x 4096, Nt = 8192, T = 1, J = 32, overlap 2, Robin p = 8, and the
# coarse grid its learned guess is trained on (same J, overlap, T and p)
SHAPE_4096 = Shape(4096, 4096, 8192, 1.0, 32, 2, kb.ROBIN, 8.0)
SHAPE_4096_COARSE = Shape(512, 512, 1024, 1.0, 32, 2, kb.ROBIN, 8.0)


def coef_matrix(seeds):
    return np.stack([inputs.coefficients(int(s)) for s in seeds]).astype(np.float64)


N_FEAT = 2 * inputs.N_COEF


def features(C):
    """Network input of coefficient rows: each coefficient as a BF16 value
    plus its remainder scaled by 2^8, so that a BF16 operand path still sees
    the coefficient to about 16 significant bits ([N][128] FP32)."""
    import torch

    c = torch.as_tensor(np.asarray(C, dtype=np.float64)).reshape(-1, inputs.N_COEF).float()
    hi = c.to(torch.bfloat16).float()
    lo = (c - hi) * 256.0
    return torch.cat([hi, lo], dim=1).contiguous()


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


def base_guess(shape: Shape, u0, base):
    """The guess a network corrects: None (zero) or Q(u0) extended in time."""
    if base == "zero":
        return None
    if base == "u0":
        return kb.u0_guess(u0, shape.nt, shape.J, shape.overlap, shape.tr, shape.p)
    raise ValueError(f"unknown base guess {base!r}")


def generate(shape: Shape, seeds, batch=128, tol=1e-10, max_iter=500, log=None, base="u0"):
    """Training targets of every seed: converged traces minus the base guess
    (FP32, [N][n_out]) and the network inputs (features(), [N][128] FP32),
    both on the GPU; plus the iteration counts."""
    import torch

    seeds = list(seeds)
    N = len(seeds)
    C = coef_matrix(seeds)
    X = features(C).cuda()
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
            b = base_guess(shape, U0[i], base)
            kb.cast_f64_f32(lam.reshape(-1), Y[b0 + i], base=None if b is None else b.reshape(-1))
            iters[b0 + i] = st.iters
        if log:
            log(f"generated {b1}/{N} traces ({time.time() - t0:.1f} s, "
                f"mean iterations {iters[:b1].mean():.1f})")
    torch.cuda.synchronize()
    return X, Y, iters


class LearnedGuess:
    """Networks + per-output scales of one problem shape.

    Stage 1 is the network (depth x hidden, GELU, optionally with the input
    skip); each further stage is a linear network (depth 0) fitted to what
    the stages before it leave over, in its own standardised units.  Two
    BF16 stages reach far below the ~2^-9 relative rounding floor of one.
    With gelu_last the linear stages (one plus `refine`) come first and the
    (depth x hidden) network is fitted last, to what they leave: placed
    earlier, it fits the training set's remainder so closely that the
    linear refinements after it have nothing left to learn that carries to
    unseen inputs.
    lambda^0 = base + sum over stages of (mean_k + std_k * net_k(x))."""

    def __init__(self, shape: Shape, hidden=512, depth=3, seed=0, base="u0", skip=True,
                 refine=0, nets=None, lead_linear=False, n_out=None, gelu_last=False):
        self.shape = shape
        self.base = base
        self.n_out = n_out or shape.n_out
        if nets is None:
            no = self.n_out
            if gelu_last:
                nets = [kb.MLP(N_FEAT, 8, 0, no, seed=seed + 100)]
                nets += [kb.MLP(N_FEAT, 8, 0, no, seed=seed + 1 + k) for k in range(refine)]
                nets += [kb.MLP(N_FEAT, hidden, depth, no, seed=seed, skip=skip)]
            else:
                # lead_linear: a linear stage first, the (depth x hidden)
                # network fitted to what it leaves over, then the refinement
                # stages
                nets = [kb.MLP(N_FEAT, 8, 0, no, seed=seed + 100)] if lead_linear else []
                nets += [kb.MLP(N_FEAT, hidden, depth, no, seed=seed, skip=skip)]
                nets += [kb.MLP(N_FEAT, 8, 0, no, seed=seed + 1 + k) for k in range(refine)]
        self.nets = nets
        self.means = []
        self.stds = []

    def _train(self, net, X, Y, epochs, batch, lr, lr_min, rng, log, tag):
        import torch

        N = X.shape[0]
        nb = max(1, N // batch)
        steps = epochs * nb
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
                tot += net.train_step(xb, yb, cur)
                k += 1
            hist.append(tot / nb)
            if log:
                log(f"{tag} epoch {ep + 1}/{epochs}: loss {hist[-1]:.4e}")
        return hist

    def fit(self, X, Y, epochs=30, batch=256, lr=1e-3, lr_min=1e-5, log=None, seed=0,
            refine_epochs=None, refine_lr=None, lrs=None, stage_epochs=None):
        """Trains every stage; Y (targets, FP32 [N][n_out]) is overwritten
        (standardised, then replaced by each stage's remainder).  Returns the
        epoch losses of all stages, in order."""
        rng = np.random.default_rng(seed)
        self.means, self.stds = [], []
        hist = []
        scale = None
        for k, net in enumerate(self.nets):
            mean, std = kb.column_stats(Y, floor=1e-6 if k == 0 else 1e-9)
            kb.standardize(Y, mean, std)
            if scale is not None:  # back to the units of lambda
                kb.mul_f32(scale, mean)
                kb.mul_f32(scale, std)
            self.means.append(mean)
            self.stds.append(std)
            ep = stage_epochs[k] if stage_epochs else (epochs if k == 0 else
                                                         (refine_epochs or epochs))
            rate = lrs[k] if lrs else (lr if k == 0 else (refine_lr or lr))
            hist += self._train(net, X, Y, ep, batch, rate, lr_min, rng, log, f"stage {k + 1}")
            if k + 1 < len(self.nets):
                for b0 in range(0, X.shape[0], batch):
                    P = net.forward(X[b0:b0 + batch].contiguous())
                    kb.axpy_f32(P, Y[b0:b0 + batch], -1.0)
            scale = std
        return hist

    def predict(self, coef, u0=None):
        """Initial traces lambda^0 (FP64 [B][2(J-1)][nt][nx]) for coefficient
        rows; u0 ([B][nv+1][nx] or [nv+1][nx], FP64 on the GPU) is needed when
        the networks correct the u0-extension guess."""
        s = self.shape
        return self.predict_flat(coef, u0).reshape(-1, 2 * (s.J - 1), s.nt, s.nx)

    def predict_flat(self, coef, u0=None):
        """The summed stages (plus the base guess) as FP64 [B][n_out]."""
        import torch

        X = features(coef).cuda()
        s = self.shape
        lam = None
        if self.base != "zero":
            if u0 is None:
                raise ValueError("this guess corrects the u0 guess: pass u0")
            u0 = u0.reshape(-1, s.nv + 1, s.nx)
            if u0.shape[0] != X.shape[0]:
                raise ValueError("one u0 per coefficient row")
            lam = torch.stack([base_guess(s, u0[i], self.base) for i in range(u0.shape[0])])
            lam = lam.reshape(X.shape[0], -1)
        for net, mean, std in zip(self.nets, self.means, self.stds):
            lam = kb.destandardize(net.forward(X), mean, std, base=lam)
        return lam

    def save(self, prefix):
        import torch

        for k, net in enumerate(self.nets):
            net.save(f"{prefix}.net{k}")
        torch.save({"means": [m.cpu() for m in self.means], "stds": [d.cpu() for d in self.stds],
                    "shape": asdict(self.shape), "base": self.base, "stages": len(self.nets)},
                   prefix + ".std.pt")

    @classmethod
    def load(cls, prefix):
        import torch

        d = torch.load(prefix + ".std.pt", weights_only=True)
        nets = [kb.MLP.load(f"{prefix}.net{k}") for k in range(d["stages"])]
        g = cls(Shape(**d["shape"]), base=d["base"], nets=nets,
                n_out=int(d["means"][0].numel()))
        g.means = [m.cuda() for m in d["means"]]
        g.stds = [x.cuda() for x in d["stds"]]
        return g


def generate_modes(shape: Shape, seeds, modes=inputs.X_FREQS, batch=64, tol=1e-10,
                   max_iter=1000, log=None):
    """Training targets of every seed as x-Fourier coefficients: the
    converged traces of each plane and level reduced to their (cos, sin)
    pairs at `modes` (the frequencies of the fields, so nothing is lost),
    FP32 [N][2(J-1) * nt * 2 len(modes)]; plus the network inputs and the
    iteration counts."""
    import torch

    seeds = list(seeds)
    N = len(seeds)
    C = coef_matrix(seeds)
    X = features(C).cuda()
    nout = 2 * (shape.J - 1) * shape.nt * 2 * len(modes)
    Y = torch.empty((N, nout), dtype=torch.float32, device="cuda")
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
            c = kb.trace_modes(lam, modes)
            kb.cast_f64_f32(c.reshape(-1), Y[b0 + i])
            iters[b0 + i] = st.iters
        del res, U0, F
        if log:
            log(f"generated {b1}/{N} coarse traces ({time.time() - t0:.1f} s, "
                f"mean iterations {iters[:b1].mean():.1f})")
    torch.cuda.synchronize()
    return X, Y, iters


class ModalGuess:
    """A learned guess trained on a coarse grid and carried to a finer one.

    The traces of fields made of the x frequencies `modes` consist of
    exactly those frequencies, so each plane and level of the coarse
    converged traces is stored as its (cos, sin) coefficient pairs.  Linear
    BF16 stages (as LearnedGuess with depth 0) map the coefficients of the
    fields to them; kfp_trace_synth evaluates the prediction on the fine
    grid (exact in x, linear in time between coarse levels).  The coarse
    grid has the fine one's J, overlap, T and transmission, so the trace
    planes correspond; what is left is the coarse grid's discretisation
    error, which the SWR iteration on the fine grid removes."""

    def __init__(self, coarse: Shape, modes=inputs.X_FREQS, refine=1, seed=0, guess=None):
        self.coarse = coarse
        self.modes = tuple(int(m) for m in modes)
        nout = 2 * (coarse.J - 1) * coarse.nt * 2 * len(self.modes)
        self.g = guess or LearnedGuess(coarse, hidden=8, depth=0, seed=seed, base="zero",
                                       skip=False, refine=refine, n_out=nout)

    def fit(self, X, Y, **kw):
        return self.g.fit(X, Y, **kw)

    def coefficients(self, coef):
        """Predicted coarse coefficients, FP64 [B][2(J-1)][ntc][2 len(modes)]."""
        c = self.coarse
        return self.g.predict_flat(coef).reshape(-1, 2 * (c.J - 1), c.nt, 2 * len(self.modes))

    def predict(self, coef, nt, nx):
        """Initial traces on the fine grid, FP64 [B][2(J-1)][nt][nx]."""
        import torch

        cc = self.coefficients(coef)
        out = torch.empty((cc.shape[0], cc.shape[1], int(nt), int(nx)), dtype=torch.float64,
                          device="cuda")
        for b in range(cc.shape[0]):
            kb.trace_synth(cc[b].contiguous(), self.modes, nt, nx, out=out[b])
        return out


def train_modal_guess(coarse: Shape, seeds, epochs=400, batch=64, lr=3e-3, refine=1, log=None):
    """Generates the coarse training solves of `seeds` and fits a ModalGuess
    to them; returns (guess, seconds generating, seconds training, mean
    coarse iterations)."""
    import torch

    t0 = time.time()
    X, Y, iters = generate_modes(coarse, seeds, log=log)
    t_gen = time.time() - t0
    g = ModalGuess(coarse, refine=refine)
    t0 = time.time()
    g.fit(X, Y, epochs=epochs, batch=batch, lr=lr, log=None)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    del X, Y
    return g, t_gen, t_train, float(iters.mean())


def evaluate(shape: Shape, seeds, guess=None, tol=1e-10, max_iter=500, log=None):
    """Iterations and wall time to tolerance for zero, u0-extension and
    learned initial traces on each seed (single solves, synchronised; the
    time of a learned run includes its inference), and the error of each
    initial guess against the converged traces (max-norm, relative to the
    traces' max-norm).  guess: one LearnedGuess (reported as "learned") or a
    dict name -> LearnedGuess."""
    import torch

    guesses = {} if guess is None else (guess if isinstance(guess, dict) else {"learned": guess})
    fm = FieldMaker(shape)
    out = {"zero": [], "u0": []}
    out.update({k: [] for k in guesses})
    C = coef_matrix(seeds)
    for i, s in enumerate(seeds):
        u0s, fs = fm.make(C[i:i + 1])
        U0 = torch.from_numpy(u0s[0]).cuda()
        F = torch.from_numpy(fs[0]).cuda()
        runs = [("zero", None), ("u0", "u0")] + [(k, g) for k, g in guesses.items()]
        ref = None
        lam_star = None
        for name, kind in runs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam0 = None
            if kind == "u0":
                lam0 = kb.u0_guess(U0, shape.nt, shape.J, shape.overlap, shape.tr, shape.p)
            elif kind is not None:
                lam0 = kind.predict(C[i], U0)[0].contiguous()
            uT, lam, st = kb.swr_solve(U0, F, shape.T, shape.nt, shape.J, shape.overlap,
                                       shape.tr, p=shape.p, tol=tol, max_iter=max_iter,
                                       lambda_init=lam0, history=False,
                                       want_lambda=lam_star is None)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if lam_star is None:
                lam_star = lam
            scale = float(lam_star.abs().max())
            gerr = float((lam_star if lam0 is None else (lam0 - lam_star)).abs().max()) / scale
            if ref is None:
                ref = uT
                err = 0.0
            else:
                err = float((uT - ref).norm() / ref.norm())
            out[name].append({"seed": int(s), "iters": st.iters, "seconds": dt, "guess_err": gerr,
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
                  "guess_err_median": float(np.median([r["guess_err"] for r in v])),
                  "max_rel_l2_vs_zero_guess": float(max(r["rel_l2_vs_zero_guess"] for r in v))}
    return res


VARIANTS = {
    # name: (depth, hidden, skip, refine, lead_linear)
    "mlp": (3, 512, False, 0, False),        # 3 x 512 GELU
    "mlp_skip": (3, 512, True, 0, False),    # 3 x 512 GELU + linear input skip
    "linear": (0, 8, False, 0, False),       # one BF16 linear layer
    "linear_x3": (0, 8, False, 2, False),    # linear + two refinement stages
    "linear_x2": (0, 8, False, 1, False),    # linear + one refinement stage
    # linear stage, the 3 x 512 GELU network on its remainder, a linear
    # refinement stage
    "linear_mlp": (3, 512, False, 1, True),
    # three linear stages, then the 3 x 512 GELU network on their remainder
    "linear_x3_mlp": (3, 512, False, 2, False, True),
}


def bench_train_steps(steps, batch=256, hidden=512, depth=3, skip=False):
    """Train steps of the network of the 256 x 256 shape on random inputs and
    targets (no solves): mean wall time per step after one warm-up step,
    for kernel profiles of the forward, backward and Adam kernels."""
    import torch

    shape = SHAPE_256
    net = kb.MLP(N_FEAT, hidden, depth, shape.n_out, seed=0, skip=skip)
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((batch, N_FEAT), generator=g, device="cuda", dtype=torch.float32)
    Y = torch.randn((batch, shape.n_out), generator=g, device="cuda", dtype=torch.float32)
    net.train_step(X, Y, 1e-4)
    # the library's copy kernel over 1 GiB: a known byte count for scaling
    # HBM counters taken on this run
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    kb.bw_probe(a, torch.empty_like(a))
    del a
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(X, Y, 1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    params = sum(net.shape(k)[0] * net.shape(k)[1] for k in range(net.layers()))
    return {"batch": batch, "hidden": hidden, "depth": depth, "skip": skip, "n_out": shape.n_out,
            "params": params, "steps": steps, "ms_per_step": dt * 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--eval", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--refine-lr", type=float, default=3e-3)
    ap.add_argument("--out", default="learned_results.json")
    ap.add_argument("--save", default=None, help="checkpoint prefix (one per variant)")
    ap.add_argument("--base", default="u0", choices=["u0", "zero"])
    ap.add_argument("--variants", default="mlp,linear_x3",
                    help="comma-separated from " + ",".join(VARIANTS))
    ap.add_argument("--orders", default="0",
                    help="evaluation in these solve orders: 0 parallel, 1 red-black")
    ap.add_argument("--scheme", choices=["fd", "fem"], default="fd",
                    help="discretisation of every solve (default fd)")
    ap.add_argument("--bench-train-steps", type=int, default=0,
                    help="only time this many train steps of the 3 x 512 network on random data")
    args = ap.parse_args()
    if args.bench_train_steps > 0:
        print(json.dumps(bench_train_steps(args.bench_train_steps, batch=args.batch)), flush=True)
        return
    kb.set_scheme(kb.FEM if args.scheme == "fem" else kb.FD)

    def log(msg):
        print(msg, flush=True)

    import torch

    shape = SHAPE_256
    t0 = time.time()
    X, Y0, iters = generate(shape, range(args.train), log=log, base=args.base)
    t_gen = time.time() - t0
    guesses, train = {}, {}
    names = [v for v in args.variants.split(",") if v]
    for k, name in enumerate(names):
        depth, hidden, skip, refine, lead, *more = VARIANTS[name]
        last = bool(more and more[0])
        Y = Y0 if k == len(names) - 1 else Y0.clone()
        g = LearnedGuess(shape, hidden=hidden, depth=depth, base=args.base, skip=skip,
                         refine=refine, lead_linear=lead, gelu_last=last)
        t0 = time.time()
        # a leading linear stage and the network after it train at --lr, the
        # refinement stages at --refine-lr; with the network last, the linear
        # stages as usual and the network at a tenth of --lr
        if last:
            lrs = [args.lr] + [args.refine_lr] * refine + [0.1 * args.lr]
        else:
            lrs = [args.lr, args.lr] + [args.refine_lr] * refine if lead else None
        hist = g.fit(X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log,
                     refine_lr=args.refine_lr, lrs=lrs)
        torch.cuda.synchronize()
        train[name] = {"seconds": time.time() - t0, "loss_history": hist,
                       "depth": depth, "hidden": hidden, "skip": skip, "refine": refine,
                       "lead_linear": lead, "gelu_last": last}
        del Y
        if args.save:
            g.save(f"{args.save}.{name}")
        guesses[name] = g
        log(f"trained {name} in {train[name]['seconds']:.1f} s")
    del X, Y0
    torch.cuda.empty_cache()
    summaries = {}
    for order in (int(x) for x in args.orders.split(",") if x):
        # the converged traces do not depend on the order: the same networks
        # serve both
        kb.set_ordering(order)
        ev = evaluate(shape, range(20000, 20000 + args.eval), guesses, log=log)
        summaries["parallel" if order == 0 else "red-black"] = summarize(ev)
    kb.set_ordering(0)
    res = {"shape": asdict(shape), "scheme": args.scheme, "base": args.base,
           "train_seeds": args.train,
           "eval_seeds": args.eval, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
           "generate_seconds": t_gen, "train_iters_mean": float(iters.mean()),
           "train": train, "summary": summaries.get("parallel") or next(iter(summaries.values())),
           "summary_by_order": summaries}
    with open(args.out, "w") as fp:
        json.dump(res, fp, indent=1)
    log(json.dumps(res["summary"]))


if __name__ == "__main__":
    main()

"""Seeded synthetic inputs for the Kolmogorov SWR solver.

This module only builds input arrays (initial data u0, source f, its time
profile s, random initial traces).  It holds none of the method's arithmetic,
so both the GPU path and the CPU oracle can be fed from it.

Fields live on the grid of Section 6.2: x_m = m/Nx (m = 0..Nx-1, periodic),
v_i = -1 + 2i/Nv (i = 0..Nv), stored row-major as [Nv+1][Nx] FP64 with x
contiguous.  Both ends v = +-1 carry u = 0.
"""
from __future__ import annotations

import math

import numpy as np

# 16 fixed Fourier x Legendre modes: index k = 4 (mx - 1) + l, mx in 1..4, l in 0..3.
N_MODES = 16
N_COEF = 4 * N_MODES  # [a (cos, f), b (sin, f), c (cos, u0), d (sin, u0)]
X_FREQS = (1, 2, 3, 4)  # the x frequencies m_x of the modes


def grid(nx: int, nv: int):
    x = np.arange(nx, dtype=np.float64) / nx
    v = -1.0 + np.arange(nv + 1, dtype=np.float64) * (2.0 / nv)
    return x, v


def legendre(l: int, v: np.ndarray) -> np.ndarray:
    if l == 0:
        return np.ones_like(v)
    if l == 1:
        return v.copy()
    if l == 2:
        return 0.5 * (3.0 * v * v - 1.0)
    if l == 3:
        return 0.5 * (5.0 * v ** 3 - 3.0 * v)
    raise ValueError(l)


def mode_basis(nx: int, nv: int):
    """Basis tensors so that field = einsum over the coefficient vector.

    Returns (Bf, Bu) of shape [32, nv+1, nx]: Bf[k] are the 16 cos and 16 sin
    modes for f, Bu[k] the same modes times (1 - v^2) for u0, so u0 vanishes
    at v = +-1.
    """
    x, v = grid(nx, nv)
    Bf = np.empty((2 * N_MODES, nv + 1, nx))
    for mx in range(1, 5):
        c = np.cos(2 * math.pi * mx * x)
        s = np.sin(2 * math.pi * mx * x)
        for l in range(4):
            k = 4 * (mx - 1) + l
            P = legendre(l, v)
            Bf[k] = P[:, None] * c[None, :]
            Bf[N_MODES + k] = P[:, None] * s[None, :]
    Bu = Bf * (1.0 - v * v)[None, :, None]
    Bu[:, 0, :] = 0.0
    Bu[:, -1, :] = 0.0
    return Bf, Bu


def coefficients(seed: int) -> np.ndarray:
    """The 64 N(0,1) mode coefficients of one seeded instance."""
    return np.random.default_rng(seed).standard_normal(N_COEF)


def fields_from_coefficients(coef: np.ndarray, nx: int, nv: int):
    """(u0, f) on the grid from a 64-vector [a, b, c, d]."""
    Bf, Bu = mode_basis(nx, nv)
    coef = np.asarray(coef, dtype=np.float64)
    f = np.tensordot(coef[: 2 * N_MODES], Bf, axes=1)
    u0 = np.tensordot(coef[2 * N_MODES:], Bu, axes=1)
    f[0, :] = 0.0
    f[-1, :] = 0.0
    return np.ascontiguousarray(u0), np.ascontiguousarray(f)


def random_fields(seed: int, nx: int, nv: int):
    """Random smooth (u0, f): 16 Fourier x Legendre modes, N(0,1) coefficients."""
    return fields_from_coefficients(coefficients(seed), nx, nv)


def manufactured(nx: int, nv: int, nt: int, T: float):
    """Manufactured solution u = sin(2 pi x) cos(pi v / 2) e^{-t}.

    Returns (u0, f, s, exact) where the source is f(t,x,v) = s(t) f(x,v) with
    s(t) = e^{-t}, sampled at t_n = n T / nt (n = 0..nt), and exact(t) gives
    the closed form on the grid.
    """
    x, v = grid(nx, nv)
    X, Vv = np.meshgrid(x, v)
    base = np.sin(2 * math.pi * X) * np.cos(math.pi * Vv / 2)
    u0 = base.copy()
    u0[0, :] = 0.0
    u0[-1, :] = 0.0
    f = np.cos(math.pi * Vv / 2) * (
        (math.pi ** 2 / 4 - 1.0) * np.sin(2 * math.pi * X) + 2 * math.pi * Vv * np.cos(2 * math.pi * X)
    )
    f[0, :] = 0.0
    f[-1, :] = 0.0
    t = np.arange(nt + 1, dtype=np.float64) * (T / nt)
    s = np.exp(-t)

    def exact(tt):
        e = base * math.exp(-tt)
        e[0, :] = 0.0
        e[-1, :] = 0.0
        return e

    return np.ascontiguousarray(u0), np.ascontiguousarray(f), s, exact


def random_traces(seed: int, J: int, nt: int, nx: int) -> np.ndarray:
    """Random initial interface data [2(J-1)][nt][nx] (error-equation tests)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((2 * (J - 1), nt, nx))


def batch_specs(n_inst: int, base_seed: int = 10_000, nt: int = 512, T: float = 0.25,
                overlap: int = 2, p: float = 4.0,
                sizes=(128, 256, 512, 1024), Js=(2, 4, 8, 16)):
    """Shapes of a batch of uneven instances: instance i draws Nx, Nv, J from
    default_rng(base_seed + i) uniformly, then its 64 field coefficients."""
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(base_seed + i)
        nx = int(rng.choice(sizes))
        nv = int(rng.choice(sizes))
        J = int(rng.choice(Js))
        coef = rng.standard_normal(N_COEF)
        out.append(dict(nx=nx, nv=nv, nt=nt, T=T, J=J, overlap=overlap, p=p, coef=coef,
                        seed=base_seed + i))
    return out

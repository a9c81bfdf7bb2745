"""Independent dense constructions used to pin the oracle (CPU, numpy only).

These build the discrete problem of Section 6.2 as ONE global linear system
over all time levels (block lower-bidiagonal in time) and solve it with
numpy.linalg.solve: a different computational route from the oracle's
column-by-column Thomas march.  Only tiny grids are used.
"""
from __future__ import annotations

import numpy as np


def transport_matrix(nx, nv, nt, T):
    """Dense matrix of the upwind x-transport acting on the interior rows
    1..nv-1 (unknown vector ordered [row][x]).  Built from the definition of
    (6.4)/(6.5): weight 1-|nu| on the cell itself, |nu| on the upwind cell."""
    hx, hv, dt = 1.0 / nx, 2.0 / nv, T / nt
    n = (nv - 1) * nx
    B = np.zeros((n, n))
    for i in range(1, nv):
        v = -1.0 + i * hv
        nu = v * dt / hx
        for m in range(nx):
            row = (i - 1) * nx + m
            B[row, row] += 1.0 - abs(nu)
            if nu > 0:
                B[row, (i - 1) * nx + (m - 1) % nx] += abs(nu)
            elif nu < 0:
                B[row, (i - 1) * nx + (m + 1) % nx] += abs(nu)
    return B


def diffusion_matrix(nx, nv, nt, T):
    """Dense (I - dt D_vv) on the interior rows with zero data at v = +-1."""
    hv, dt = 2.0 / nv, T / nt
    r = dt / hv ** 2
    n = (nv - 1) * nx
    A = np.zeros((n, n))
    for i in range(1, nv):
        for m in range(nx):
            row = (i - 1) * nx + m
            A[row, row] = 1.0 + 2.0 * r
            if i - 1 >= 1:
                A[row, (i - 2) * nx + m] = -r
            if i + 1 <= nv - 1:
                A[row, i * nx + m] = -r
    return A


def spacetime_mono(u0, f, T, nt, s=None):
    """All time levels U^1..U^nt of the monodomain scheme from one dense
    space-time solve of  A U^{n+1} - B U^n = dt s_{n+1} f  (n = 0..nt-1).
    Returns an array [nt+1][nv+1][nx] (level 0 = u0 with zeroed ends)."""
    nv, nx = u0.shape[0] - 1, u0.shape[1]
    dt = T / nt
    A = diffusion_matrix(nx, nv, nt, T)
    B = transport_matrix(nx, nv, nt, T)
    n = (nv - 1) * nx
    N = n * nt
    M = np.zeros((N, N))
    rhs = np.zeros(N)
    x0 = u0[1:nv].reshape(-1)
    fi = f[1:nv].reshape(-1)
    for k in range(nt):
        M[k * n:(k + 1) * n, k * n:(k + 1) * n] = A
        sk = 1.0 if s is None else s[k + 1]
        rhs[k * n:(k + 1) * n] = dt * sk * fi
        if k == 0:
            rhs[:n] += B @ x0
        else:
            M[k * n:(k + 1) * n, (k - 1) * n:k * n] = -B
    X = np.linalg.solve(M, rhs)
    out = np.zeros((nt + 1, nv + 1, nx))
    out[0] = u0
    out[0, 0] = 0.0
    out[0, -1] = 0.0
    for k in range(nt):
        out[k + 1, 1:nv] = X[k * n:(k + 1) * n].reshape(nv - 1, nx)
    return out


def interface_data(U, a, b, nv, transmission, p, q=None):
    """Interface variables (6.7) of a glued field history U [nt+1][nv+1][nx]
    for the partition a, b: plane 2j = Q_2 U at a_{j+1}, plane 2j+1 = Q_1 U at
    b_j, levels 1..nt.  Q = I (Dirichlet) or Q_1 = p + d/dv, Q_2 = q - d/dv
    (q = p unless given) with one-sided differences pointing into the
    subdomain that receives it."""
    q = p if q is None else q
    hv = 2.0 / nv
    J = len(a)
    nt = U.shape[0] - 1
    nx = U.shape[2]
    lam = np.zeros((2 * (J - 1), nt, nx))
    for j in range(J - 1):
        al, be = a[j + 1], b[j]
        for n in range(1, nt + 1):
            if transmission == 0:
                lam[2 * j, n - 1] = U[n, al]
                lam[2 * j + 1, n - 1] = U[n, be]
            else:
                lam[2 * j, n - 1] = q * U[n, al] - (U[n, al + 1] - U[n, al]) / hv
                lam[2 * j + 1, n - 1] = p * U[n, be] + (U[n, be] - U[n, be - 1]) / hv
    return lam


def interface_data_nonoverlap(U, f, T, nv, a, b, p, q=None, s=None):
    """Interface variables of the non-overlapping decomposition (a_{j+1} =
    b_j: the neighbours share the node) that make the glued field history U
    [nt+1][nv+1][nx] satisfy each subdomain's half-cell row at the shared node.
    The row of the subdomain below (Robin condition (p + d/dv) u = lambda_1,
    so the flux through the interface is lambda_1 - p u) times 2 dt/h_v:
        (1 + 2r + 2 dt p / h_v) U_b - 2r U_{b-1} = (T U^{n-1})_b + dt s f_b + 2 dt/h_v lambda_1
    and above (flux q u - lambda_2):
        (1 + 2r + 2 dt q / h_v) U_a - 2r U_{a+1} = (T U^{n-1})_a + dt s f_a + 2 dt/h_v lambda_2.
    Solved here for lambda from U; plane 2j = lambda_2 (for j+1), 2j+1 =
    lambda_1 (for j), levels 1..nt."""
    q = p if q is None else q
    nt = U.shape[0] - 1
    nx = U.shape[2]
    hx, hv, dt = 1.0 / nx, 2.0 / nv, T / nt
    r = dt / hv ** 2
    hc = 2.0 * dt / hv
    J = len(a)

    def upwind(row, i):
        nu = (-1.0 + i * hv) * dt / hx
        if nu > 0:
            nb = np.roll(row, 1)  # value at m-1
        elif nu < 0:
            nb = np.roll(row, -1)  # value at m+1
        else:
            nb = row
        return (1.0 - abs(nu)) * row + abs(nu) * nb

    lam = np.zeros((2 * (J - 1), nt, nx))
    for j in range(J - 1):
        c = b[j]
        assert a[j + 1] == c
        for n in range(1, nt + 1):
            sn = 1.0 if s is None else s[n]
            tu = upwind(U[n - 1, c], c)
            src = dt * sn * f[c]
            lam[2 * j + 1, n - 1] = ((1 + 2 * r + hc * p) * U[n, c] - 2 * r * U[n, c - 1]
                                     - tu - src) / hc
            lam[2 * j, n - 1] = ((1 + 2 * r + hc * q) * U[n, c] - 2 * r * U[n, c + 1]
                                 - tu - src) / hc
    return lam


# ---------------------------------------------------------------------------
# The finite-element scheme of Section 6.2 (linear elements, Neumann ends,
# diffusion then transport), assembled here from its definitions.
# ---------------------------------------------------------------------------
def hat(i, v, nv):
    """Nodal basis function phi_i of the linear elements on v_i = -1 + i h."""
    h = 2.0 / nv
    return max(0.0, 1.0 - abs(v - (-1.0 + i * h)) / h)


def hat_slope(i, v, nv):
    """phi_i' inside an element (v strictly between nodes)."""
    h = 2.0 / nv
    vi = -1.0 + i * h
    if abs(v - vi) >= h:
        return 0.0
    return 1.0 / h if v < vi else -1.0 / h


def fem_matrices(nv, lo=0, hi=None):
    """Mass and stiffness matrices (6.3) on nodes 0..nv, each entry summed
    element by element with Simpson's rule (exact for these integrands, the
    Remark after (6.5)).  The slope is evaluated at interior points only.
    lo, hi: only the elements inside [v_lo, v_hi] (a subdomain's own)."""
    h = 2.0 / nv
    hi = nv if hi is None else hi
    M = np.zeros((nv + 1, nv + 1))
    S = np.zeros((nv + 1, nv + 1))
    for e in range(lo, hi):
        v0, v1 = -1.0 + e * h, -1.0 + (e + 1) * h
        vm = 0.5 * (v0 + v1)
        for i in (e, e + 1):
            for j in (e, e + 1):
                M[i, j] += h / 6.0 * (hat(i, v0, nv) * hat(j, v0, nv)
                                      + 4.0 * hat(i, vm, nv) * hat(j, vm, nv)
                                      + hat(i, v1, nv) * hat(j, v1, nv))
                # the slopes are constant on the element: Simpson with the
                # midpoint value three times over (interior points only)
                S[i, j] += h * hat_slope(i, vm, nv) * hat_slope(j, vm, nv)
    return M, S


def transport_matrix_all(nx, nv, nt, T):
    """Upwind transport (6.4)/(6.5) on every node row 0..nv, ordered [row][x]."""
    hx, hv, dt = 1.0 / nx, 2.0 / nv, T / nt
    n = (nv + 1) * nx
    B = np.zeros((n, n))
    for i in range(nv + 1):
        nu = (-1.0 + i * hv) * dt / hx
        for m in range(nx):
            row = i * nx + m
            B[row, row] += 1.0 - abs(nu)
            if nu > 0:
                B[row, i * nx + (m - 1) % nx] += abs(nu)
            elif nu < 0:
                B[row, i * nx + (m + 1) % nx] += abs(nu)
    return B


def spacetime_fem_mono(u0, f, T, nt, s=None):
    """The finite-element scheme as one dense space-time system in the
    diffusion-stage unknowns W^1..W^nt (all nodes, all x):
        (M/dt + S) W^1 = M/dt (u0 + dt s_1 f),
        (M/dt + S) W^{n+1} - M/dt Tr W^n = M s_{n+1} f,
    and U^nt = Tr W^nt.  Returns (W [nt+1][nv+1][nx] with W[0] = u0, uT)."""
    nv, nx = u0.shape[0] - 1, u0.shape[1]
    dt = T / nt
    Mv, Sv = fem_matrices(nv)
    I = np.eye(nx)
    A = np.kron(Mv / dt + Sv, I)
    Bm = np.kron(Mv / dt, I)
    Tr = transport_matrix_all(nx, nv, nt, T)
    n = (nv + 1) * nx
    N = n * nt
    K = np.zeros((N, N))
    rhs = np.zeros(N)
    fv = f.reshape(-1)
    for k in range(nt):
        sk = 1.0 if s is None else s[k + 1]
        K[k * n:(k + 1) * n, k * n:(k + 1) * n] = A
        rhs[k * n:(k + 1) * n] = Bm @ (dt * sk * fv)
        if k == 0:
            rhs[:n] += Bm @ u0.reshape(-1)
        else:
            K[k * n:(k + 1) * n, (k - 1) * n:k * n] = -Bm @ Tr
    X = np.linalg.solve(K, rhs)
    W = np.zeros((nt + 1, nv + 1, nx))
    W[0] = u0
    for k in range(nt):
        W[k + 1] = X[k * n:(k + 1) * n].reshape(nv + 1, nx)
    uT = (Tr @ W[nt].reshape(-1)).reshape(nv + 1, nx)
    return W, uT


def fem_interface_data(W, u0, f, T, a, b, nv, transmission, p, q=None, s=None):
    """Interface variables that make the glued diffusion-stage history W
    [nt+1][nv+1][nx] satisfy every subdomain's interface row of the
    finite-element scheme: the RECEIVING subdomain's row at its interface
    node (one element, natural Robin condition), solved for lambda.  Times
    dt/h, with G^n = Tr W^n + dt s f (G^0 = u0 + dt s f) and r = dt/h^2:
      below beta:  (1/6)[(W_{b-1}-G_{b-1}) + 2(W_b-G_b)] + r(W_b-W_{b-1}) + dt/h p W_b = dt/h lambda_1
      above alpha: (1/6)[2(W_a-G_a) + (W_{a+1}-G_{a+1})] + r(W_a-W_{a+1}) + dt/h q W_a = dt/h lambda_2
    Dirichlet: the node values.  Plane 2j = lambda_2 (for j+1), 2j+1 =
    lambda_1 (for j), levels 1..nt."""
    q = p if q is None else q
    nt = W.shape[0] - 1
    nx = W.shape[2]
    hv, dt = 2.0 / nv, T / nt
    r, k = dt / hv ** 2, dt / hv
    Tr = transport_matrix_all(nx, nv, nt, T)
    J = len(a)
    lam = np.zeros((2 * (J - 1), nt, nx))
    for n in range(1, nt + 1):
        sn = 1.0 if s is None else s[n]
        U = u0 if n == 1 else (Tr @ W[n - 1].reshape(-1)).reshape(nv + 1, nx)
        G = U + dt * sn * f
        Wn = W[n]
        for j in range(J - 1):
            al, be = a[j + 1], b[j]
            if transmission == 0:
                lam[2 * j, n - 1] = Wn[al]
                lam[2 * j + 1, n - 1] = Wn[be]
                continue
            row_b = ((Wn[be - 1] - G[be - 1]) + 2 * (Wn[be] - G[be])) / 6.0 \
                + r * (Wn[be] - Wn[be - 1]) + k * p * Wn[be]
            row_a = (2 * (Wn[al] - G[al]) + (Wn[al + 1] - G[al + 1])) / 6.0 \
                + r * (Wn[al] - Wn[al + 1]) + k * q * Wn[al]
            lam[2 * j + 1, n - 1] = row_b / k
            lam[2 * j, n - 1] = row_a / k
    return lam

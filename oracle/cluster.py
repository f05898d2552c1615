"""Cluster environments (Sec. 5): CU_0 separable boundaries and n x n windows.

Test infrastructure only (see the package docstring).

CU_0 (Sec. 5.1, figs. SepEnv1/SepEnv2): the part of the norm network above a
row cut is approximated by a boundary MPO of bond D' = 1, i.e. one positive
D x D matrix sigma_c per cut vertical bond (ket leg x bra leg).  It is found
by ALS over the sites of the row being absorbed; because the other local
tensors enter only through their norms, the norm matrix of each local problem
is a positive multiple of the identity and the update is sigma_c ~ b_c, with
b_c the network contracted around the site.  Starting from positive sigma
this stays positive.  The start used here is identity/sqrt(D) (positive; the
paper suggests X^T X with random X), the sweeps alternate direction and stop
when no sigma_c changed by more than ``tol`` in Frobenius norm.

Windows (Sec. 5.2-5.3): outside a cluster the environment is separable and
inside it the sandwich contraction with bond D' runs as usual.  The cluster
around site (i, j) is the n x n window of rows/columns
[i - ceil(n/2) + 1, i + floor(n/2)] clipped to the lattice (reading); its cut
legs are closed by the separable boundaries of the four directions (corners
drop out at D' = 1).  A window's outputs are <S^z> of its centre site and the
bond energies of the centre's right and down bonds.
"""
import numpy as np

from .boundary import Lattice, flip_vertical, transpose_lattice
from .api import env_boundary, expect, DEFAULT_SEED, DEFAULT_HALFSWEEPS

EIN = dict(optimize=True)


def _row_double_layer(sig_up, A):
    """P[l,m,d,g,r,s] = sum sig_up[u,v] A[p,l,u,r,d] A[p,m,v,s,g]."""
    return np.einsum("uv,plurd,pmvsg->lmdgrs", sig_up, A, A, **EIN)


def _unit(X):
    return X / np.sqrt(np.sum(X * X))


def separable_row(sig_up, Arow, lam, rho, tol=1e-14, max_sweeps=500):
    """One CU_0 absorption: sigma'_c for the down legs of ``Arow``."""
    Lc = len(Arow)
    P = [_row_double_layer(sig_up[c], Arow[c]) for c in range(Lc)]
    sig = [np.eye(A.shape[4]) / np.sqrt(A.shape[4]) for A in Arow]
    e = [None] * (Lc + 1)
    f = [None] * (Lc + 1)
    e[0], f[Lc] = lam, rho
    for c in range(Lc - 1, 0, -1):
        f[c] = _unit(np.einsum("lmdgrs,dg,rs->lm", P[c], sig[c], f[c + 1], **EIN))
    sweeps, delta = 0, np.inf
    while sweeps < max_sweeps:
        old = [s.copy() for s in sig]
        for c in range(Lc):                                   # left to right
            b = np.einsum("lm,lmdgrs,rs->dg", e[c], P[c], f[c + 1], **EIN)
            sig[c] = _unit(b)
            if c < Lc - 1:
                e[c + 1] = _unit(np.einsum("lm,lmdgrs,dg->rs", e[c], P[c], sig[c], **EIN))
        for c in range(Lc - 1, -1, -1):                       # right to left
            b = np.einsum("lm,lmdgrs,rs->dg", e[c], P[c], f[c + 1], **EIN)
            sig[c] = _unit(b)
            if c > 0:
                f[c] = _unit(np.einsum("lmdgrs,dg,rs->lm", P[c], sig[c], f[c + 1], **EIN))
        sweeps += 1
        delta = max(float(np.sqrt(np.sum((s - o) ** 2))) for s, o in zip(sig, old))
        if delta <= tol:
            break
    return sig, sweeps, delta


def separable_top(lat, tol=1e-14, max_sweeps=500):
    """sig[r][c], r = 0..Lr-2: CU_0 boundary of rows 0..r on the down legs of row r."""
    out = []
    up = list(lat.tau)
    for r in range(lat.rows - 1):
        up, _, _ = separable_row(up, lat.A[r], lat.lam[r], lat.rho[r], tol, max_sweeps)
        out.append(up)
    return out


class SeparableEnv:
    """CU_0 boundaries of the four directions of a lattice."""

    def __init__(self, lat, tol=1e-14, max_sweeps=500):
        Lr, Lc = lat.rows, lat.cols
        self.lat = lat
        self.top = separable_top(lat, tol, max_sweeps)
        self.bot = separable_top(flip_vertical(lat), tol, max_sweeps)
        tl = transpose_lattice(lat)
        self.left = separable_top(tl, tol, max_sweeps)
        self.right = separable_top(flip_vertical(tl), tol, max_sweeps)
        self.Lr, self.Lc = Lr, Lc

    def above(self, r0, c):
        """Closing of the up legs of row r0 at column c (rows < r0 contracted)."""
        return self.lat.tau[c] if r0 == 0 else self.top[r0 - 1][c]

    def below(self, r1, c):
        """Closing of the down legs of row r1 (rows > r1 contracted)."""
        return self.lat.beta[c] if r1 == self.Lr - 1 else self.bot[self.Lr - 2 - r1][c]

    def leftof(self, r, c0):
        """Closing of the left legs of (r, c0) (columns < c0 contracted)."""
        return self.lat.lam[r] if c0 == 0 else self.left[c0 - 1][r]

    def rightof(self, r, c1):
        return self.lat.rho[r] if c1 == self.Lc - 1 else self.right[self.Lc - 2 - c1][r]


def window_bounds(i, n, L):
    lo = max(0, i - (n + 1) // 2 + 1)
    hi = min(L - 1, i + n // 2)
    return lo, hi


def window_lattice(sep, r0, r1, c0, c1):
    lat = sep.lat
    A = [[lat.A[r][c] for c in range(c0, c1 + 1)] for r in range(r0, r1 + 1)]
    lam = [sep.leftof(r, c0) for r in range(r0, r1 + 1)]
    rho = [sep.rightof(r, c1) for r in range(r0, r1 + 1)]
    tau = [sep.above(r0, c) for c in range(c0, c1 + 1)]
    beta = [sep.below(r1, c) for c in range(c0, c1 + 1)]
    return Lattice(A, lam, rho, tau, beta)


def cluster_env(lat, n, chi, halfsweeps=DEFAULT_HALFSWEEPS, seed=DEFAULT_SEED,
                tol=1e-14, max_sweeps=500, sites=None, sep=None):
    """Per-site window results: dict (i, j) -> (sz, bond_right, bond_down).
    ``sep``: CU_0 boundaries of ``lat`` from an earlier call (else built here)."""
    sep = sep if sep is not None else SeparableEnv(lat, tol, max_sweeps)
    Lr, Lc = lat.rows, lat.cols
    out = {}
    for (i, j) in (sites if sites is not None else [(i, j) for i in range(Lr) for j in range(Lc)]):
        r0, r1 = window_bounds(i, n, Lr)
        c0, c1 = window_bounds(j, n, Lc)
        win = window_lattice(sep, r0, r1, c0, c1)
        res = expect(env_boundary(win, chi, halfsweeps, seed), rows=[i - r0])
        ci, cj = i - r0, j - c0
        right = res["bond_h"][ci, cj] if j < c1 else np.nan
        down = res["bond_v"][ci, cj] if i < r1 else np.nan
        out[(i, j)] = (res["sz"][ci, cj], right, down)
    return out, sep

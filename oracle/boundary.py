"""Boundary-MPS row absorption (the "sandwich contraction" of Sec. 2).

Test infrastructure only (see the package docstring).

The norm network <psi|psi> of an open-boundary PEPS is contracted from the top
row down (and, mirrored, from the bottom row up): the contracted part is an
MPS whose local tensors carry a ket and a bra leg (the "boundary MPO" of
fig. Sandwich (b)).  Absorbing one more double-layer row is an MPS-MPO product
whose bond grows by D^2; it is replaced by the best MPS of bond D' (= chi
here), found by alternating least squares (ALS) with a QR gauge, which is what
the paper states gives the optimum of the original method (Sec. 2 and the
end of Sec. 4).  The leading cost is O(D^4 D'^3) + O(d D^6 D'^2) per
absorption (fig. Sandwich caption); the contraction order below follows it.

Conventions (readings of the paper, identical on the GPU side)
-----------------------------------------------------------------
* Site tensor A[p, l, u, r, d]; "u" points to row 0.  Real entries, so the bra
  is the same tensor as the ket (no conjugation).
* A boundary tensor is T[a, k, b, a'] (left bond, ket leg, bra leg, right bond).
* A ``Lattice`` carries closing matrices for the cut legs: lam[r] on the left
  legs of row r, rho[r] on the right legs, tau[c] on the up legs of row 0 and
  beta[c] on the down legs of the last row.  For a whole lattice every
  closing is the 1x1 matrix [[1]]; for a cluster window they are the CU_0
  separable boundary matrices (Sec. 5.1-5.2).
* Bond caps: chi_c = min(chi, chi_in_c * Dr_c^2, prod_{c'<=c} Dd^2,
  prod_{c'>c} Dd^2), made consistent so that chi_c <= chi_{c-1} Dd_c^2 and
  chi_{c-1} <= Dd_c^2 chi_c.  If every cap equals the product bond the row is
  absorbed exactly; otherwise by ALS.
* ALS: start tensors from SplitMix64 (``splitmix``), right-canonical start by
  LQ, ``halfsweeps`` alternating half-sweeps (first one left to right), QR
  gauge with non-negative R diagonal, then the centre tensor is normalised
  and 0.5*log(omega) is added to the boundary's log-scale, omega being the
  squared norm of the final centre tensor.
* Stopping: with ``tol`` = 0 exactly ``halfsweeps`` half-sweeps run.  With
  ``tol`` > 0 the sweep goes on past ``halfsweeps`` (at least 2) until the
  squared centre norm settles, |omega_h - omega_(h-1)| <= tol * omega_h, or
  ``max_halfsweeps`` have run (the row is then marked not converged).
  omega is the squared overlap of the fit with the exact product, which is
  stationary at the optimum: the rule fixes omega to about tol and the
  tensors only to about sqrt(tol) (directions of tiny weight in the boundary
  go on rotating long after omega and the observables have settled).
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import splitmix

EIN = dict(optimize=True)


@dataclass
class Lattice:
    """Sites A[r][c] (each (d, Dl, Du, Dr, Dd)) plus cut-leg closings."""
    A: List[List[np.ndarray]]
    lam: List[np.ndarray] = field(default_factory=list)
    rho: List[np.ndarray] = field(default_factory=list)
    tau: List[np.ndarray] = field(default_factory=list)
    beta: List[np.ndarray] = field(default_factory=list)

    @property
    def rows(self):
        return len(self.A)

    @property
    def cols(self):
        return len(self.A[0])


def whole_lattice(A):
    """A whole open-boundary lattice: every cut leg has dimension 1."""
    Lr, Lc = len(A), len(A[0])
    for r in range(Lr):
        for c in range(Lc):
            d, Dl, Du, Dr, Dd = A[r][c].shape
            if c + 1 < Lc:
                assert Dr == A[r][c + 1].shape[1], "horizontal bond mismatch"
            if r + 1 < Lr:
                assert Dd == A[r + 1][c].shape[2], "vertical bond mismatch"
    one = np.ones((1, 1))
    for r in range(Lr):
        assert A[r][0].shape[1] == 1 and A[r][Lc - 1].shape[3] == 1
    for c in range(Lc):
        assert A[0][c].shape[2] == 1 and A[Lr - 1][c].shape[4] == 1
    return Lattice([list(row) for row in A], [one] * Lr, [one] * Lr,
                   [one] * Lc, [one] * Lc)


def flip_vertical(lat):
    """Mirror the lattice top<->bottom (rows reversed, u and d legs swapped)."""
    A = [[t.transpose(0, 1, 4, 3, 2) for t in row] for row in reversed(lat.A)]
    return Lattice(A, lat.lam[::-1], lat.rho[::-1], list(lat.beta), list(lat.tau))


def transpose_lattice(lat):
    """Swap rows and columns (l<->u, r<->d); left/right become top/bottom."""
    Lr, Lc = lat.rows, lat.cols
    A = [[lat.A[r][c].transpose(0, 2, 1, 4, 3) for r in range(Lr)] for c in range(Lc)]
    return Lattice(A, list(lat.tau), list(lat.beta), list(lat.lam), list(lat.rho))


def qr_pos(M):
    """Reduced QR with non-negative diagonal of R (unique for full column rank)."""
    Q, R = np.linalg.qr(M)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s, R * s[:, None]


def bond_caps(chi, chi_prod, Dd):
    """Target bonds of the new boundary at the Lc-1 inner cuts (see module doc)."""
    Lc = len(Dd)
    caps = []
    for c in range(Lc - 1):
        left = int(np.prod([Dd[k] ** 2 for k in range(c + 1)], dtype=object))
        right = int(np.prod([Dd[k] ** 2 for k in range(c + 1, Lc)], dtype=object))
        caps.append(min(chi, chi_prod[c], left, right))
    full = [1] + caps + [1]
    for c in range(Lc):
        full[c + 1] = min(full[c + 1], full[c] * Dd[c] ** 2)
    for c in reversed(range(Lc)):
        full[c] = min(full[c], full[c + 1] * Dd[c] ** 2)
    return full[1:-1]


# --- the four-stage chain of one site (indices: x new-left, a old-left,
#     l/m ket/bra left legs, u/v up legs, p physical, r/s right legs,
#     d/g down legs, e old-right, y new-right) ---------------------------------

def chain_left(E, T, A):
    """Y[x,e,r,d,s,g] = sum E[x,a,l,m] T[a,u,v,e] A[p,l,u,r,d] A[p,m,v,s,g]."""
    Y = np.einsum("xalm,auve->xlmuve", E, T, **EIN)
    Y = np.einsum("xlmuve,plurd->xmveprd", Y, A, **EIN)
    return np.einsum("xmveprd,pmvsg->xerdsg", Y, A, **EIN)


def chain_right(F, T, A):
    """Y[y,a,l,d,m,g] = sum F[y,e,r,s] T[a,u,v,e] A[p,l,u,r,d] A[p,m,v,s,g]."""
    Y = np.einsum("yers,auve->yrsauv", F, T, **EIN)
    Y = np.einsum("yrsauv,plurd->ysavpld", Y, A, **EIN)
    return np.einsum("ysavpld,pmvsg->yaldmg", Y, A, **EIN)


def site_tensor(E, T, A, F):
    """ALS local solution N[x,d,g,y] = E . (T A A) . F (identity norm matrix)."""
    return np.einsum("xerdsg,yers->xdgy", chain_left(E, T, A), F, **EIN)


def env_left(E, T, A, Q):
    return np.einsum("xerdsg,xdgy->yers", chain_left(E, T, A), Q, **EIN)


def env_right(F, T, A, Q):
    return np.einsum("yaldmg,xdgy->xalm", chain_right(F, T, A), Q, **EIN)


def product_site(T, A):
    """Exact MPS-MPO product tensor P[a,l,m,d,g,e,r,s]."""
    return np.einsum("auve,plurd,pmvsg->almdgers", T, A, A, **EIN)


@dataclass
class AbsorbInfo:
    exact: bool
    omegas: list
    bonds: list
    converged: bool = True


def absorb_row(T, Arow, lam, rho, chi, halfsweeps, seed, side, row, tol=0.0, max_halfsweeps=None):
    """T_new ~ T . row, returns (T_new, dlog, info); T_new has unit norm."""
    Lc = len(Arow)
    Dr = [t.shape[3] for t in Arow]
    Dd = [t.shape[4] for t in Arow]
    chi_in = [T[c].shape[3] for c in range(Lc - 1)]
    chi_prod = [chi_in[c] * Dr[c] ** 2 for c in range(Lc - 1)]
    caps = bond_caps(chi, chi_prod, Dd)
    if caps == chi_prod:
        return _absorb_exact(T, Arow, lam, rho, Dd)
    return _absorb_als(T, Arow, lam, rho, caps, Dd, halfsweeps, seed, side, row, tol, max_halfsweeps)


def _absorb_exact(T, Arow, lam, rho, Dd):
    Lc = len(Arow)
    X = []
    for c in range(Lc):
        P = product_site(T[c], Arow[c])
        a, l, m, d, g, e, r, s = P.shape
        if c == 0:
            P = np.einsum("almdgers,lm->adgers", P, lam, **EIN)[:, None, None]
            l = m = 1
        if c == Lc - 1:
            P = np.einsum("almdgers,rs->almdge", P, rho, **EIN)[..., None, None]
            r = s = 1
        X.append(P.reshape(a * l * m, d, g, e * r * s))
    # left-canonicalise by QR, the norm ends up in the last tensor
    for c in range(Lc - 1):
        xl, d, g, xr = X[c].shape
        Q, R = qr_pos(X[c].reshape(xl * d * g, xr))
        X[c] = Q.reshape(xl, d, g, Q.shape[1])
        X[c + 1] = np.einsum("xy,ydgz->xdgz", R, X[c + 1], **EIN)
    omega = float(np.sum(X[-1] ** 2))
    X[-1] = X[-1] / np.sqrt(omega)
    return X, 0.5 * np.log(omega), AbsorbInfo(True, [omega], [t.shape[3] for t in X[:-1]])


def _absorb_als(T, Arow, lam, rho, caps, Dd, halfsweeps, seed, side, row, tol=0.0, max_halfsweeps=None):
    Lc = len(Arow)
    bonds = [1] + list(caps) + [1]
    X = []
    for c in range(Lc):
        shape = (bonds[c], Dd[c], Dd[c], bonds[c + 1])
        vals = splitmix.uniform(seed, splitmix.als_stream(side, row, c), int(np.prod(shape)))
        X.append(vals.reshape(shape))
    # right-canonical start: X[c] = L Q with orthonormal rows (LQ = QR of the transpose)
    for c in range(Lc - 1, 0, -1):
        xl, d, g, xr = X[c].shape
        Q, R = qr_pos(X[c].reshape(xl, d * g * xr).T)
        X[c] = Q.T.reshape(xl, d, g, xr)
        X[c - 1] = np.einsum("adgx,yx->adgy", X[c - 1], R, **EIN)
    E = [None] * (Lc + 1)
    F = [None] * (Lc + 1)
    Dl0, DrL = Arow[0].shape[1], Arow[-1].shape[3]
    E[0] = lam.reshape(1, 1, Dl0, Dl0)
    F[Lc] = rho.reshape(1, 1, DrL, DrL)
    for c in range(Lc - 1, 0, -1):
        F[c] = env_right(F[c + 1], T[c], Arow[c], X[c])
    omegas = []
    adaptive = tol > 0.0
    h_min = max(halfsweeps, 2) if adaptive else halfsweeps
    h_max = max(max_halfsweeps or h_min, h_min) if adaptive else halfsweeps
    converged = not adaptive
    for h in range(h_max):
        if h % 2 == 0:                       # left to right
            for c in range(Lc):
                N = site_tensor(E[c], T[c], Arow[c], F[c + 1])
                if c < Lc - 1:
                    xl, d, g, xr = N.shape
                    Q, _ = qr_pos(N.reshape(xl * d * g, xr))
                    X[c] = Q.reshape(xl, d, g, xr)
                    E[c + 1] = env_left(E[c], T[c], Arow[c], X[c])
                else:
                    X[c] = N
        else:                                # right to left
            for c in range(Lc - 1, -1, -1):
                N = site_tensor(E[c], T[c], Arow[c], F[c + 1])
                if c > 0:
                    xl, d, g, xr = N.shape
                    Q, _ = qr_pos(N.reshape(xl, d * g * xr).T)
                    X[c] = Q.T.reshape(xl, d, g, xr)
                    F[c] = env_right(F[c + 1], T[c], Arow[c], X[c])
                else:
                    X[c] = N
        omegas.append(float(np.sum(N ** 2)))
        if adaptive and h + 1 >= h_min and abs(omegas[-1] - omegas[-2]) <= tol * omegas[-1]:
            converged = True
            break
    centre = Lc - 1 if len(omegas) % 2 == 1 else 0
    X[centre] = X[centre] / np.sqrt(omegas[-1])
    return X, 0.5 * np.log(omegas[-1]), AbsorbInfo(False, omegas, list(caps), converged)


def mps_overlap(X, Y):
    """<X|Y> of two boundaries of one lattice row, each tensor [a, k, b, a']
    with (k, b) taken as one physical index: the trace tr(X^T Y) of the two
    boundary MPOs (Sec. 5.2 measures boundary fidelity with it)."""
    E = np.ones((1, 1))
    for x, y in zip(X, Y):
        E = np.einsum("xy,xkbz,ykbw->zw", E, x, y, **EIN)
    return float(E[0, 0])


def boundary_fidelity(X, Y):
    """|<X|Y>| / sqrt(<X|X> <Y|Y>)."""
    return abs(mps_overlap(X, Y)) / np.sqrt(mps_overlap(X, X) * mps_overlap(Y, Y))


def trivial_boundary(closing_list):
    """The bond-1 product MPS made of the closing matrices of one side."""
    return [np.asarray(s, dtype=np.float64).reshape(1, s.shape[0], s.shape[1], 1)
            for s in closing_list]


def top_boundaries(lat, chi, halfsweeps=4, seed=0, side=0, tol=0.0, max_halfsweeps=None):
    """Boundaries T_r (rows 0..r absorbed) for r = -1 .. Lr-2.

    Returns a list ``out`` with out[r+1] = (tensors, log_scale, info).
    """
    out = [(trivial_boundary(lat.tau), 0.0, None)]
    T, s = out[0][0], 0.0
    for r in range(lat.rows - 1):
        T, dlog, info = absorb_row(T, lat.A[r], lat.lam[r], lat.rho[r], chi,
                                   halfsweeps, seed, side, r, tol, max_halfsweeps)
        s += dlog
        out.append((T, s, info))
    return out

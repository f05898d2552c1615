"""One imaginary-time full-update Trotter step of a PEPS (Secs. 2 and 5.2),
plain and slow.  Test infrastructure only: it pins the library's evolution
driver and is not used by it.

The step applies exp(-tau h) (h = S.S of eq. HeisenbergH on one bond) to
every nearest-neighbour bond, in four sets of disjoint bonds: horizontal
bonds with even, then odd, left column; vertical bonds with even, then odd,
upper row.  For one set, the environment of the current state is built
once (row boundaries for horizontal bonds, column boundaries for vertical
ones).  The two new tensors of a bond fit G psi (Sec. 2): with the second
one fixed at S2, S1 minimises || psi' - G psi || (the linear problem
S1 N1 = b1 of the bond's pair environment), then S2 with the new S1, for
``als`` alternations.  N is symmetrised and inverted on its eigenvectors
whose eigenvalue exceeds ``cutoff`` times the largest (the problem is
singular along directions the environment does not see).  Each new tensor
is rescaled to unit largest entry (the state's norm is not evolved).  After
the fit the shared bond is rebalanced: the product of the two tensors over
that bond is split again by a singular value decomposition, the square roots
of the singular values going to each side.  The bond dimension stays fixed.
"""
import numpy as np
import scipy.linalg

from . import api
from .spin import bond_matrix


def gate(tau):
    """exp(-tau h) on one bond as G[s1', s2', s1, s2] (outputs first)."""
    return scipy.linalg.expm(-tau * bond_matrix()).reshape(2, 2, 2, 2)


def fit_solve(N, b, cutoff):
    """S with S N = b, N symmetrised and pseudo-inverted above the cutoff."""
    N = 0.5 * (N + N.T)
    w, V = np.linalg.eigh(N)
    keep = w > cutoff * np.max(w)
    Ninv = V[:, keep] @ np.diag(1.0 / w[keep]) @ V[:, keep].T
    return b @ Ninv


def rebalance(S1, S2, vertical):
    """S1 (left or upper site) and S2 with the same product over their shared
    bond, split by SVD with sqrt of the singular values on each side."""
    leg1, leg2 = (4, 2) if vertical else (3, 1)   # S1's down/right leg, S2's up/left leg
    a = np.moveaxis(S1, leg1, 4)                   # (.., bond)
    b = np.moveaxis(S2, leg2, 0)                   # (bond, ..)
    D = a.shape[4]
    U, s, Vh = np.linalg.svd(a.reshape(-1, D) @ b.reshape(D, -1), full_matrices=False)
    U, s, Vh = U[:, :D], s[:D], Vh[:D, :]
    if len(s) < D:   # a product of rank below D: the missing bond values are zero
        k = D - len(s)
        U = np.hstack([U, np.zeros((U.shape[0], k))])
        Vh = np.vstack([Vh, np.zeros((k, Vh.shape[1]))])
        s = np.concatenate([s, np.zeros(k)])
    h = np.sqrt(s)
    new1 = np.moveaxis((U * h[None, :]).reshape(a.shape), 4, leg1)
    new2 = np.moveaxis((h[:, None] * Vh).reshape(b.shape), 0, leg2)
    return new1, new2


def update_bond_set(A, bonds, vertical, G, chi, als, cutoff):
    """Fit every bond of one set of disjoint bonds from one environment."""
    partner = [(r + 1, c) if vertical else (r, c + 1) for (r, c) in bonds]
    env = api.env_columns(A, chi) if vertical else api.env_boundary(A, chi)
    S1 = [A[r][c].copy() for (r, c) in bonds]
    S2 = [A[r][c].copy() for (r, c) in partner]
    for _ in range(als):
        for which in (0, 1):
            for k, (r, c) in enumerate(bonds):
                fit = api.bond_fit_vertical if vertical else api.bond_fit
                N1, b1, N2, b2 = fit(env, r, c, G, S1[k], S2[k])
                if which == 0:
                    new = fit_solve(N1, b1, cutoff).reshape(S1[k].shape)
                    S1[k] = new / np.max(np.abs(new))
                else:
                    new = fit_solve(N2, b2, cutoff).reshape(S2[k].shape)
                    S2[k] = new / np.max(np.abs(new))
    for k, ((r, c), (r2, c2)) in enumerate(zip(bonds, partner)):
        t1, t2 = rebalance(S1[k], S2[k], vertical)
        A[r][c] = t1 / np.max(np.abs(t1))
        A[r2][c2] = t2 / np.max(np.abs(t2))


def trotter_step(A, tau, chi, als=3, cutoff=1e-12):
    """One Trotter step on a copy of the site list A; returns the new list."""
    A = [[np.array(t, dtype=np.float64) for t in row] for row in A]
    Lr, Lc = len(A), len(A[0])
    G = gate(tau)
    for vertical in (False, True):
        for parity in (0, 1):
            if vertical:
                bonds = [(r, c) for r in range(parity, Lr - 1, 2) for c in range(Lc)]
            else:
                bonds = [(r, c) for r in range(Lr) for c in range(parity, Lc - 1, 2)]
            if bonds:
                update_bond_set(A, bonds, vertical, G, chi, als, cutoff)
    return A

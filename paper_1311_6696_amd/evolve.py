"""Imaginary-time evolution of a PEPS by full updates (Secs. 2 and 5.2), a
consumer of the library's environments.

Each Trotter step applies exp(-tau S_l.S_m) on every nearest-neighbour bond
in four sets of disjoint bonds (horizontal with even / odd left column,
vertical with even / odd upper row).  For one set, one environment of the
current state is built (with column boundaries for the vertical sets), and
for every bond of the set the two new site tensors are found by alternating
least squares on the fit of G psi (Sec. 2): with the second site held at S2,
S1 solves S1 N1 = b1, then S2 solves S2 N2 = b2 with the new S1; N and b
come from the library (``peps_bond_fit``: the bond's pair environment from
the fixed boundaries, the substitutes in place of the sites), the K x K
solves run here on the host with a relative eigenvalue cutoff; the two new
tensors are then split symmetrically over their shared bond (SVD of their
product, the square root of the singular values to each side: the bond's
gauge, which the fit leaves free, would otherwise drift and spoil the
conditioning of later fits) and rescaled to unit largest entry.  The bond dimension D stays
fixed: the truncation of the evolved state is the fit itself.  With
boundaries at lossless chi the energies are exact expectation values of the
evolved PEPS, so they are bounded below by the exact ground-state energy.
"""
import numpy as np

from . import binding


def heisenberg_gate(tau):
    """exp(-tau S.S) for two spins 1/2 as G[p, P, q, Q]."""
    sz = np.diag([0.5, -0.5])
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    h = np.kron(sz, sz) + 0.5 * (np.kron(sp, sp.T) + np.kron(sp.T, sp))
    ev, U = np.linalg.eigh(h)
    return (U @ np.diag(np.exp(-tau * ev)) @ U.T).reshape(2, 2, 2, 2)


def _solve(N, b, cutoff):
    """A' with A' N = b, N symmetrised, eigenvalues below cutoff * max dropped."""
    Ns = 0.5 * (N + N.T)
    w, V = np.linalg.eigh(Ns)
    keep = w > cutoff * w.max()
    inv = (V[:, keep] / w[keep]) @ V[:, keep].T
    return b @ inv


def energy_per_site(sess, A, chi):
    env = sess.env_boundary([binding.to_device(A)], chi)[0]
    r = sess.expect([env])[0]
    env.free()
    return float(np.sum(r["bond_h"]) + np.sum(r["bond_v"])) / (len(A) * len(A[0]))


def full_update(sess, A, tau, steps, chi, cutoff=1e-12, als=3, every=1, log=None, sequential=False,
                balance=True):
    """Evolve the site list A (numpy, (d, Dl, Du, Dr, Dd) each) for `steps`
    Trotter steps of size tau with `als` alternating sweeps per bond;
    sequential: a new environment for every bond instead of one per bond set;
    balance: after each bond's fit, split the product of its two tensors over
    the shared bond symmetrically (SVD, same product).
    Returns (A, [(step, energy per site)])."""
    import torch
    A = [[np.array(t, dtype=np.float64) for t in row] for row in A]
    Lr, Lc = len(A), len(A[0])
    g = torch.as_tensor(heisenberg_gate(tau), device="cuda")
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), device="cuda")
    trace = []
    for step in range(steps):
        for direction, parity in ((0, 0), (0, 1), (1, 0), (1, 1)):
            if direction == 0:
                bonds = [(r, c) for r in range(Lr) for c in range(parity, Lc - 1, 2)]
            else:
                bonds = [(r, c) for r in range(parity, Lr - 1, 2) for c in range(Lc)]
            for group in ([[b] for b in bonds] if sequential else [bonds]):
                _update_bonds(sess, A, group, direction, g, chi, als, cutoff, dev, balance)
        if (step + 1) % every == 0 or step + 1 == steps:
            e = energy_per_site(sess, A, chi)
            trace.append((step + 1, e))
            if log:
                log(f"step {step + 1}: energy per site {e:.8f}")
    return A, trace


def _balance(S1, S2, direction):
    """Rebalance the shared bond of S1 (left or upper) and S2 without changing
    their product: SVD of the product over the bond, sqrt(s) to each side."""
    ax1, ax2 = (3, 1) if direction == 0 else (4, 2)    # S1's right/down leg, S2's left/up leg
    t1 = np.moveaxis(S1, ax1, -1)
    t2 = np.moveaxis(S2, ax2, 0)
    D = t1.shape[-1]
    M = t1.reshape(-1, D) @ t2.reshape(D, -1)
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    U, s, Vh = U[:, :D], s[:D], Vh[:D]
    r = np.sqrt(s)
    n1 = np.moveaxis((U * r).reshape(t1.shape), -1, ax1)
    n2 = np.moveaxis((r[:, None] * Vh).reshape(t2.shape), 0, ax2)
    return n1, n2


def _update_bonds(sess, A, bonds, direction, g, chi, als, cutoff, dev, balance=False):
    """Alternating fits of the disjoint bonds `bonds` from one environment."""
    other = [(r, c + 1) if direction == 0 else (r + 1, c) for r, c in bonds]
    env = sess.env_boundary([binding.to_device(A)], chi, columns=direction == 1)[0]
    S1 = [A[r][c].copy() for r, c in bonds]
    S2 = [A[r][c].copy() for r, c in other]
    for _ in range(als):
        for side in (0, 1):
            got, _ = sess.bond_fit([(env, r, c, direction, g, dev(s1), dev(s2))
                                    for (r, c), s1, s2 in zip(bonds, S1, S2)])
            for k, (n1, b1, n2, b2) in enumerate(got):
                N, b = (n1, b1) if side == 0 else (n2, b2)
                S = S1 if side == 0 else S2
                new = _solve(N.cpu().numpy(), b.cpu().numpy(), cutoff).reshape(S[k].shape)
                S[k] = new / np.abs(new).max()
    env.free()
    for k, ((r, c), (r2, c2)) in enumerate(zip(bonds, other)):
        s1, s2 = _balance(S1[k], S2[k], direction) if balance else (S1[k], S2[k])
        A[r][c], A[r2][c2] = s1 / np.abs(s1).max(), s2 / np.abs(s2).max()


def neel_start(Lr, Lc, D, noise=1e-2, seed=0):
    """Neel product state with small random virtual entries (bond D)."""
    rng = np.random.default_rng(seed)
    A = []
    for r in range(Lr):
        row = []
        for c in range(Lc):
            shape = (2, 1 if c == 0 else D, 1 if r == 0 else D, 1 if c == Lc - 1 else D, 1 if r == Lr - 1 else D)
            t = noise * rng.standard_normal(shape)
            t[((r + c) % 2, 0, 0, 0, 0)] += 1.0
            row.append(t)
        A.append(row)
    return A

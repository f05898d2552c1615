"""Imaginary-time evolution of a PEPS by full updates (Secs. 2 and 5.2), a
consumer of the library's environments.

Each Trotter step applies exp(-tau S_l.S_m) on every nearest-neighbour bond
in four sets of disjoint bonds (horizontal with even / odd left column,
vertical with even / odd upper row), each set in two passes: the first pass
refits the first site of every bond, the second the other site.  In a pass,
one environment of the current state gives, through the C ABI, the norm
environment N and the right-hand side b of the refitted site of every bond
(the row sandwiches for horizontal bonds, the column sandwiches for
vertical ones); the site is replaced by the solution of A' N = b, the ALS
local problem of fitting G psi with only that site free (computed here on the
host from the K x K matrices with a relative eigenvalue cutoff), rescaled
to unit largest entry.  Refitting one site of a bond at a time keeps each
update an exact least-squares fit; refitting both from one environment would
let each site take up the whole change of the bond.  The second pass fits
the gate applied to the state after the first pass, so each bond sees the
gate twice per step (an effective step of 2 tau).  The bond dimension D stays fixed: the truncation of
the evolved state is the optimisation itself.  With boundaries at lossless
chi the energies are exact expectation values of the evolved PEPS, so they
are bounded below by the exact ground-state energy.
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


def full_update(sess, A, tau, steps, chi, cutoff=1e-12, every=1, log=None):
    """Evolve the site list A (numpy, (d, Dl, Du, Dr, Dd) each) for `steps`
    Trotter steps of size tau; returns (A, [(step, energy per site)])."""
    import torch
    A = [[np.array(t, dtype=np.float64) for t in row] for row in A]
    Lr, Lc = len(A), len(A[0])
    g = torch.as_tensor(heisenberg_gate(tau), device="cuda")
    trace = []
    for step in range(steps):
        for direction, parity in ((0, 0), (0, 1), (1, 0), (1, 1)):
            if direction == 0:
                bonds = [(r, c) for r in range(Lr) for c in range(parity, Lc - 1, 2)]
            else:
                bonds = [(r, c) for r in range(parity, Lr - 1, 2) for c in range(Lc)]
            if not bonds:
                continue
            other = [(r, c + 1) if direction == 0 else (r + 1, c) for r, c in bonds]
            for side in (0, 1):
                env = sess.env_boundary([binding.to_device(A)], chi, columns=direction == 1)[0]
                sites = bonds if side == 0 else other
                Ns, _ = sess.site_env([(env, r, c, direction) for r, c in sites])
                bs, _ = sess.bond_env([(env, r, c, g, direction) for r, c in bonds])
                env.free()
                for k, (rr, cc) in enumerate(sites):
                    N = Ns[k][0].cpu().numpy()
                    b = bs[k][side].cpu().numpy()
                    new = _solve(N, b, cutoff).reshape(A[rr][cc].shape)
                    A[rr][cc] = new / np.abs(new).max()
        if (step + 1) % every == 0 or step + 1 == steps:
            e = energy_per_site(sess, A, chi)
            trace.append((step + 1, e))
            if log:
                log(f"step {step + 1}: energy per site {e:.8f}")
    return A, trace


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

"""Exact references used only to pin the oracle (test infrastructure).

* ``statevector`` contracts a small PEPS into its 2^N amplitudes (the map F of
  fig. PEPS applied to every configuration), sites in row-major order with the
  first site as the slowest index; ``sv_observables`` then evaluates
  <psi|psi>, <S^z_i> and nearest-neighbour <S_i . S_j> directly.
* ``closed_network`` contracts a tiny double-layer network with closing
  matrices on its cut legs by one ``einsum`` (no boundary MPS involved).
* ``heisenberg_ground_energy`` is a Lanczos (ARPACK) ground state of
  eq. (HeisenbergH) on an open L x L lattice, which the paper quotes for
  4 x 4 in its appendix.
"""
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .spin import BOND_TERMS, SZ, ID


def statevector(A):
    Lr, Lc = len(A), len(A[0])
    psi = np.ones((1, 1) + tuple(A[0][c].shape[2] for c in range(Lc)))
    for r in range(Lr):
        for c in range(Lc):
            x = np.tensordot(psi, A[r][c], axes=([1, 2 + c], [1, 2]))
            nv = Lc - 1
            vs = list(range(1, 1 + nv))
            order = [0, 1 + nv, 2 + nv] + vs[:c] + [3 + nv] + vs[c:]
            x = x.transpose(order)
            psi = x.reshape((x.shape[0] * x.shape[1],) + x.shape[2:])
    return psi.reshape(-1)


def _apply(psi, N, site, O):
    t = psi.reshape((2,) * N)
    t = np.moveaxis(np.tensordot(O, t, axes=([1], [site])), 0, site)
    return t.reshape(-1)


def sv_observables(A):
    Lr, Lc = len(A), len(A[0])
    N = Lr * Lc
    psi = statevector(A)
    nrm = float(psi @ psi)
    sz = np.zeros((Lr, Lc))
    for r in range(Lr):
        for c in range(Lc):
            sz[r, c] = psi @ _apply(psi, N, r * Lc + c, SZ) / nrm

    def bond(i, j):
        tot = 0.0
        for w, O1, O2 in BOND_TERMS:
            tot += w * (psi @ _apply(_apply(psi, N, j, O2), N, i, O1))
        return tot / nrm

    bh = np.array([[bond(r * Lc + c, r * Lc + c + 1) for c in range(Lc - 1)] for r in range(Lr)])
    bv = np.array([[bond(r * Lc + c, (r + 1) * Lc + c) for c in range(Lc)] for r in range(Lr - 1)])
    return dict(norm=nrm, sz=sz, bond_h=bh.reshape(Lr, Lc - 1), bond_v=bv.reshape(Lr - 1, Lc))


def closed_network(lat, ops=None):
    """Contract the double-layer network of a tiny Lattice with its closings.

    ``ops`` maps (r, c) -> operator on that site's ket.  Returns the scalar.
    """
    Lr, Lc = lat.rows, lat.cols
    ops = ops or {}
    letters = iter(
        [chr(x) for x in range(ord("a"), ord("z") + 1)] + [chr(x) for x in range(ord("A"), ord("Z") + 1)])
    hk = {}  # horizontal bond (r, c)-(r, c+1) -> (ket letter, bra letter)
    vk = {}
    for r in range(Lr):
        for c in range(Lc + 1):
            hk[(r, c)] = (next(letters), next(letters))
    for r in range(Lr + 1):
        for c in range(Lc):
            vk[(r, c)] = (next(letters), next(letters))
    terms, operands = [], []
    for r in range(Lr):
        for c in range(Lc):
            p = next(letters)
            A = lat.A[r][c]
            ket = A if (r, c) not in ops else np.einsum("pq,qlurd->plurd", ops[(r, c)], A)
            l, u, rr, d = hk[(r, c)], vk[(r, c)], hk[(r, c + 1)], vk[(r + 1, c)]
            terms.append(p + l[0] + u[0] + rr[0] + d[0])
            operands.append(ket)
            terms.append(p + l[1] + u[1] + rr[1] + d[1])
            operands.append(A)
    for r in range(Lr):
        terms.append("".join(hk[(r, 0)]))
        operands.append(lat.lam[r])
        terms.append("".join(hk[(r, Lc)]))
        operands.append(lat.rho[r])
    for c in range(Lc):
        terms.append("".join(vk[(0, c)]))
        operands.append(lat.tau[c])
        terms.append("".join(vk[(Lr, c)]))
        operands.append(lat.beta[c])
    return float(np.einsum(",".join(terms) + "->", *operands, optimize="greedy"))


def closed_network_observables(lat):
    Lr, Lc = lat.rows, lat.cols
    Z = closed_network(lat)
    sz = np.array([[closed_network(lat, {(r, c): SZ}) / Z for c in range(Lc)] for r in range(Lr)])

    def bond(a, b):
        return sum(w * closed_network(lat, {a: O1, b: O2}) for w, O1, O2 in BOND_TERMS) / Z

    bh = np.array([[bond((r, c), (r, c + 1)) for c in range(Lc - 1)] for r in range(Lr)])
    bv = np.array([[bond((r, c), (r + 1, c)) for c in range(Lc)] for r in range(Lr - 1)])
    return dict(Z=Z, sz=sz, bond_h=bh.reshape(Lr, Lc - 1), bond_v=bv.reshape(Lr - 1, Lc))


def heisenberg_hamiltonian(Lr, Lc):
    N = Lr * Lc

    def op(O, i):
        m = sp.identity(1, format="csr")
        for k in range(N):
            m = sp.kron(m, sp.csr_matrix(O if k == i else ID), format="csr")
        return m

    H = sp.csr_matrix((2 ** N, 2 ** N))
    bonds = [(r * Lc + c, r * Lc + c + 1) for r in range(Lr) for c in range(Lc - 1)]
    bonds += [(r * Lc + c, (r + 1) * Lc + c) for r in range(Lr - 1) for c in range(Lc)]
    for i, j in bonds:
        for w, O1, O2 in BOND_TERMS:
            H = H + w * (op(O1, i) @ op(O2, j))
    return H, bonds


def heisenberg_ground_energy(Lr, Lc):
    H, _ = heisenberg_hamiltonian(Lr, Lc)
    w = spla.eigsh(H, k=1, which="SA", tol=1e-12)[0]
    return float(w[0])


def all_configs(N):
    return itertools.product(range(2), repeat=N)

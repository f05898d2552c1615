"""Spin-1/2 operators for the Heisenberg model of eq. (HeisenbergH), Sec. 3.

H = sum over nearest-neighbour pairs <l,m> of S_l . S_m with S = sigma/2 and
unit coupling.  Physical index 0 is spin up (S^z = +1/2).  The bond term is
written in the ladder form  S^z S^z + (S^+ S^- + S^- S^+)/2, which equals
S^x S^x + S^y S^y + S^z S^z.
"""
import numpy as np

SZ = np.array([[0.5, 0.0], [0.0, -0.5]])
SP = np.array([[0.0, 1.0], [0.0, 0.0]])   # raises index 1 -> 0
SM = SP.T.copy()
ID = np.eye(2)

# (weight, operator on the first site, operator on the second site)
BOND_TERMS = ((1.0, SZ, SZ), (0.5, SP, SM), (0.5, SM, SP))


def bond_matrix():
    """The 4x4 bond Hamiltonian h = S.S in the basis |s1 s2>."""
    return sum(w * np.kron(a, b) for w, a, b in BOND_TERMS)

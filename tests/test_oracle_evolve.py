"""Pins of the oracle's full-update Trotter step (``oracle/evolve.py``)
against what the mathematics fixes: a two-site lattice is fitted exactly
(its bond holds any two-spin state), so one bond update must return G psi
for any gate G, including a random, non-symmetric one that catches a
transposed gate or swapped sites; the identity gate leaves a state
unchanged; imaginary time lowers the energy of a Neel state."""
import numpy as np
import pytest

from oracle import evolve, exact
from paper_1311_6696_amd.inputs import make_peps


def _overlap(a, b):
    """|<a|b>| / (|a| |b|) of two state vectors."""
    return abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))


def _neel(Lr, Lc, D, noise, seed):
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


@pytest.mark.parametrize("vertical", [False, True])
def test_two_site_bond_update_is_exact_for_any_gate(vertical):
    rng = np.random.default_rng(3 + vertical)
    G = rng.standard_normal((2, 2, 2, 2))
    A = make_peps(2, 1, 3, "normal_unit", 11) if vertical else make_peps(1, 2, 3, "normal_unit", 11)
    psi = exact.statevector(A)
    want = G.reshape(4, 4) @ psi
    B = [[t.copy() for t in row] for row in A]
    evolve.update_bond_set(B, [(0, 0)], vertical, G, 16, 2, 1e-13)
    assert _overlap(exact.statevector(B), want) > 1 - 1e-12


def test_identity_gate_keeps_the_state():
    A = make_peps(2, 3, 2, "normal_unit", 5)
    psi = exact.statevector(A)
    B = evolve.trotter_step(A, 0.0, 64)
    assert _overlap(exact.statevector(B), psi) > 1 - 1e-11


def test_trotter_step_lowers_the_energy():
    A = _neel(3, 3, 2, 0.1, 0)
    e = []
    for _ in range(3):
        sv = exact.sv_observables(A)
        e.append(np.sum(sv["bond_h"]) + np.sum(sv["bond_v"]))   # normalised expectation values
        A = evolve.trotter_step(A, 0.1, 64)
    assert e[1] < e[0] - 1e-3 and e[2] < e[1]

"""Imaginary-time full updates driven through the site and bond
environments (a consumer of the library) on the 4x4 Heisenberg model."""
import sys

import numpy as np
import pytest

from oracle import evolve as oracle_evolve
from oracle import exact
from paper_1311_6696_amd import binding, evolve

pytestmark = pytest.mark.gpu
E0_4X4 = -0.57432544   # exact ground-state energy per site (App. A), pinned in the oracle tests


def test_full_update_lowers_energy_and_respects_the_bound():
    """From a Neel start, D = 2 at lossless chi: the energy per site falls
    steadily well below the Neel value and never below the exact ground
    state (the energies are exact expectation values of the evolved PEPS);
    the final state's energy agrees with its brute-force state vector."""
    print("4x4 D=2 full update", flush=True)
    sess = binding.Session(0)
    A = evolve.neel_start(4, 4, 2, 1e-1, 0)
    e_start = evolve.energy_per_site(sess, A, 16)
    A, trace = evolve.full_update(sess, A, 0.1, 10, 16, cutoff=1e-10, every=2)
    es = [e for _, e in trace]
    assert abs(e_start + 0.375) < 0.05
    assert es[-1] < -0.53
    assert all(b <= a + 1e-3 for a, b in zip(es, es[1:]))   # imaginary time lowers the energy
    assert all(e > E0_4X4 - 1e-9 for e in es)
    sv = exact.sv_observables(A)
    e_sv = (np.sum(sv["bond_h"]) + np.sum(sv["bond_v"])) / 16
    assert abs(e_sv - es[-1]) < 1e-10


def test_trotter_step_matches_oracle_step():
    """One Trotter step of the driver (library environments and fits on the
    GPU, solves and rebalancing on the host) against the oracle's step from
    the same 3x3 D=2 Neel start at lossless chi: the two states agree up to
    normalisation (the bond gauges may differ by signs), so do the energies."""
    print("3x3 D=2 one Trotter step against the oracle", flush=True)
    sess = binding.Session(0)
    A0 = evolve.neel_start(3, 3, 2, 1e-1, 4)
    A_gpu, _ = evolve.full_update(sess, A0, 0.1, 1, 64, cutoff=1e-12, als=3)
    A_ref = oracle_evolve.trotter_step(A0, 0.1, 64, als=3, cutoff=1e-12)
    a, b = exact.statevector(A_gpu), exact.statevector(A_ref)
    ov = abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))
    ea, eb = (exact.sv_observables(X) for X in (A_gpu, A_ref))
    e_gpu = np.sum(ea["bond_h"]) + np.sum(ea["bond_v"])
    e_ref = np.sum(eb["bond_h"]) + np.sum(eb["bond_v"])
    print(f"  1 - overlap {1 - ov:.2e}, energy {e_gpu:.12f} vs {e_ref:.12f}", flush=True)
    assert 1 - ov < 1e-10
    assert abs(e_gpu - e_ref) < 1e-9

"""Imaginary-time full updates driven through the site and bond
environments (a consumer of the library) on the 4x4 Heisenberg model."""
import sys

import numpy as np
import pytest

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

"""Host-side pieces of the imaginary-time driver (no GPU): the gate and the
bond rebalancing."""
import numpy as np
import pytest

from oracle import spin
from paper_1311_6696_amd import evolve


def test_heisenberg_gate_is_exp_of_the_bond_operator():
    """exp(-tau S.S): singlet eigenvalue e^{3 tau/4}, triplet e^{-tau/4}; G
    symmetric; G(a) G(b) = G(a + b)."""
    for tau in (0.0, 0.05, 0.3):
        G = evolve.heisenberg_gate(tau).reshape(4, 4)
        assert np.abs(G - G.T).max() < 1e-14
        w = np.sort(np.linalg.eigvalsh(G))
        np.testing.assert_allclose(w, np.sort([np.exp(0.75 * tau)] + [np.exp(-0.25 * tau)] * 3), rtol=1e-13)
    Ga, Gb, Gab = (evolve.heisenberg_gate(t).reshape(4, 4) for t in (0.1, 0.2, 0.3))
    np.testing.assert_allclose(Ga @ Gb, Gab, atol=1e-14)
    h = sum(w_ * np.kron(a, b) for w_, a, b in spin.BOND_TERMS)
    np.testing.assert_allclose((np.eye(4) - evolve.heisenberg_gate(1e-6).reshape(4, 4)) / 1e-6, h, atol=1e-5)


@pytest.mark.parametrize("direction", [0, 1])
def test_bond_rebalancing_keeps_the_product(direction):
    rng = np.random.default_rng(direction)
    S1 = rng.standard_normal((2, 3, 2, 4, 4)) * np.array([1e3, 1, 1e-3, 1])[None, None, None, :, None] \
        if direction == 0 else rng.standard_normal((2, 3, 2, 4, 4))
    S2 = rng.standard_normal((2, 4, 3, 2, 2)) if direction == 0 else rng.standard_normal((2, 3, 4, 2, 2))
    n1, n2 = evolve._balance(S1, S2, direction)
    spec = "plurd,qrURD->pluqURdD" if direction == 0 else "plurd,qLdRD->plurqLRD"
    np.testing.assert_allclose(np.einsum(spec, n1, n2), np.einsum(spec, S1, S2), atol=1e-10)
    # the shared bond carries equal norms on both sides afterwards
    ax1, ax2 = (3, 1) if direction == 0 else (4, 2)
    a = np.linalg.norm(np.moveaxis(n1, ax1, 0).reshape(4, -1), axis=1)
    b = np.linalg.norm(np.moveaxis(n2, ax2, 0).reshape(4, -1), axis=1)
    np.testing.assert_allclose(a, b, rtol=1e-10)

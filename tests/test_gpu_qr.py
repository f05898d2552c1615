"""The gauge QR (peps_qr) against the oracle's QR with a non-negative R
diagonal, through the C ABI.

Full-rank blocks: Q and R agree with the oracle's factors to a bound that
grows with the condition number (two backward-stable factorizations of the
same matrix differ by about kappa * eps), and Q is orthonormal, R upper
triangular with R_ii >= 0 and A = QR to working precision.  Rank-deficient
and very ill-conditioned blocks have no unique factors: there only the
properties are checked.  These blocks drive the tall-block CholeskyQR2
kernel into its Householder fallback.
"""
import sys

import numpy as np
import pytest

from oracle.boundary import qr_pos
from paper_1311_6696_amd import binding

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sess():
    return binding.Session(0)


def block(m, n, kappa, seed):
    """m x n matrix with singular values spread geometrically from 1 to
    1/kappa (kappa = 1: a plain Gaussian block)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((m, n))
    if kappa == 1:
        return G
    U, _ = np.linalg.qr(G)
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.geomspace(1.0, 1.0 / kappa, n)
    return (U * s) @ V.T


def check_props(A, Q, R, tol=1e-12):
    m, n = A.shape
    scale = max(np.abs(A).max(), 1e-300)
    assert np.abs(Q.T @ Q - np.eye(n)).max() < tol, "Q not orthonormal"
    assert np.abs(np.tril(R, -1)).max() == 0.0, "R not upper triangular"
    assert np.all(np.diag(R) >= 0.0), "negative R diagonal"
    assert np.abs(Q @ R - A).max() < tol * scale, "A != QR"


def run(sess, mats, inplace=False):
    import torch
    dev = [torch.as_tensor(np.ascontiguousarray(A), device="cuda") for A in mats]
    out = sess.qr(dev, inplace=inplace)
    torch.cuda.synchronize()
    return [(Q.cpu().numpy(), R.cpu().numpy()) for Q, R in out]


# CholeskyQR2 variants (n <= 16 / 32, m <= 256 / 512) with ragged edges,
# then register Householder, TSQR and the streaming kernel.
SHAPES = [(512, 32), (256, 32), (512, 16), (256, 16), (130, 32), (200, 17), (512, 1), (333, 9),
          (16, 16), (64, 8), (100, 40), (1000, 32), (700, 24), (300, 100)]


@pytest.mark.parametrize("m,n", SHAPES)
def test_qr_matches_oracle(sess, m, n):
    say(f"qr {m}x{n} gaussian")
    A = block(m, n, 1, 7000 + m + n)
    (Q, R), = run(sess, [A])
    Qr, Rr = qr_pos(A)
    assert np.abs(Q - Qr).max() < 1e-12
    assert np.abs(R - Rr).max() < 1e-12 * np.abs(Rr).max()
    check_props(A, Q, R)


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_qr_conditioned(sess, kappa):
    say(f"qr 512x32 kappa={kappa:g}")
    A = block(512, 32, kappa, 42)
    (Q, R), = run(sess, [A])
    Qr, Rr = qr_pos(A)
    assert np.abs(Q - Qr).max() < 1e-14 * kappa * 32
    assert np.abs(R - Rr).max() < 1e-14 * kappa * 32 * np.abs(Rr).max()
    check_props(A, Q, R)


def test_qr_column_scaling(sess):
    """Columns of very different norms (well conditioned once scaled)."""
    say("qr 512x32 column scales 1e-6..1e6")
    A = block(512, 32, 1, 5) * np.geomspace(1e-6, 1e6, 32)
    (Q, R), = run(sess, [A])
    Qr, Rr = qr_pos(A)
    assert np.abs(Q - Qr).max() < 1e-11
    check_props(A, Q, R)


@pytest.mark.parametrize("case", ["kappa1e12", "zero_column", "repeated_column", "rank4"])
def test_qr_fallback_blocks(sess, case):
    say(f"qr fallback {case}")
    if case == "kappa1e12":
        A = block(512, 32, 1e12, 3)
    elif case == "zero_column":
        A = block(512, 32, 1, 4)
        A[:, 7] = 0.0
    elif case == "repeated_column":
        A = block(256, 32, 1, 5)
        A[:, 20] = A[:, 3]
    else:
        rng = np.random.default_rng(6)
        A = rng.standard_normal((512, 4)) @ rng.standard_normal((4, 16))
    (Q, R), = run(sess, [A])
    check_props(A, Q, R)


def test_qr_batched_mixed_and_strided(sess):
    """One call with blocks of different shapes (one launch group), some
    given as transposed views, and an in-place call."""
    import torch
    say("qr batched mixed shapes, strided, in place")
    mats = [block(512, 32, 1, 11), block(16, 16, 1, 12), block(300, 20, 1e3, 13), block(512, 32, 1e12, 14)]
    dev = [torch.as_tensor(A, device="cuda") for A in mats]
    dev[2] = torch.as_tensor(np.ascontiguousarray(mats[2].T), device="cuda").t()   # column-major view
    out = sess.qr(dev)
    torch.cuda.synchronize()
    for i, (A, (Q, R)) in enumerate(zip(mats, out)):
        Q, R = Q.cpu().numpy(), R.cpu().numpy()
        check_props(A, Q, R)
        if i < 3:
            Qr, Rr = qr_pos(A)
            assert np.abs(Q - Qr).max() < 1e-10
    # in place: Q overwrites A
    A = block(512, 32, 1, 15)
    t = torch.as_tensor(A, device="cuda")
    (Q, R), = sess.qr([t], inplace=True)
    torch.cuda.synchronize()
    assert Q.data_ptr() == t.data_ptr()
    Qr, Rr = qr_pos(A)
    assert np.abs(t.cpu().numpy() - Qr).max() < 1e-12
    # repeated call gives the same bits
    (Q2, R2), = run(sess, [A])
    (Q3, R3), = run(sess, [A])
    assert np.array_equal(Q2, Q3) and np.array_equal(R2, R3)

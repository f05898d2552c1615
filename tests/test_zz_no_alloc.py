"""peps_qr_noalloc (all workspace in the library's fixed per-GPU array)
against peps_qr: the same blocks give the same factors bit for bit, on two
calls in a row (the second smaller, so it runs over what the first left in
the shared array), for every QR route (CholeskyQR2, register Householder,
the TSQR tree, the streaming kernel); a request too large for the array is
refused before anything runs."""
import sys

import numpy as np
import pytest

from paper_1311_6696_amd import binding

pytestmark = pytest.mark.gpu

LIMIT = 32 << 20   # PEPS_QR_NOALLOC_BYTES


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def blocks_of(torch, shapes, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return [torch.randn(m, n, generator=g, dtype=torch.float64).cuda() for m, n in shapes]


def run(sess, mats, noalloc):
    torch = sess.torch
    out, raw = [], []
    for A in mats:
        m, n = A.shape
        Q = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
        R = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
        raw.append((A.data_ptr(), A.stride(0), A.stride(1), Q.data_ptr(), Q.stride(0), Q.stride(1),
                    R.data_ptr(), R.stride(0), R.stride(1), m, n))
        out.append((Q, R))
    sess.ctx.qr_raw(raw, noalloc=noalloc)
    torch.cuda.synchronize()
    return [(Q.cpu().numpy(), R.cpu().numpy()) for Q, R in out]


@pytest.fixture(scope="module")
def sess():
    return binding.Session(0)


def test_noalloc_qr_matches_qr_on_two_calls(sess):
    """Calls in a row, each smaller than the one before, one per QR route
    (a batched call takes the route of its largest block): the TSQR tree,
    the streaming kernel, CholeskyQR2, register Householder."""
    torch = sess.torch
    calls = [[(2592, 72), (2592, 72), (1296, 36)],
             [(300, 100), (130, 100)],
             [(512, 32), (512, 32), (200, 20)],
             [(64, 8)]]
    for k, shapes in enumerate(calls):
        say(f"noalloc QR call {k}: {shapes}")
        mats = blocks_of(torch, shapes, 11 + k)
        ref = run(sess, mats, False)
        got = run(sess, mats, True)
        for (Qr, Rr), (Qg, Rg), A, (m, n) in zip(ref, got, mats, shapes):
            assert np.array_equal(Qr, Qg), (k, m, n)
            assert np.array_equal(Rr, Rg), (k, m, n)
            A = A.cpu().numpy()
            assert np.abs(Qg @ Rg - A).max() < 1e-12 * np.abs(A).max() * np.sqrt(m)
            assert np.abs(Qg.T @ Qg - np.eye(n)).max() < 1e-12


def test_noalloc_qr_refuses_oversized_request(sess):
    torch = sess.torch
    say("noalloc QR oversized")
    m, n = 8192, 512     # streaming workspace alone: 2*m*n doubles = 64 MiB > the array
    assert 16 * m * n > LIMIT
    A = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    Q = torch.full((m, n), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.PepsError) as ei:
        sess.ctx.qr_raw([(A.data_ptr(), n, 1, Q.data_ptr(), n, 1, None, 0, 0, m, n)], noalloc=True)
    assert ei.value.code == -2
    torch.cuda.synchronize()
    assert bool(torch.all(Q == 7.0))   # nothing was written

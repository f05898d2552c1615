"""Error paths of the C ABI on the GPU: invalid requests, non-finite inputs,
the workspace cap and the ALS convergence flag.  Each failing call must
return its status, leave every output handle NULL and write no result."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1311_6696_amd import binding
from paper_1311_6696_amd.inputs import make_peps

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sess():
    return binding.Session(0)


SENTINEL = 0x5EED


def call_boundary(sess, states, opts):
    """Raw peps_env_boundary with out[] pre-filled by a sentinel; returns
    (status, out handles, error text)."""
    lib = sess.ctx.lib
    n = len(states)
    arr = (binding.State * n)(*[s.struct() for s in states])
    out = (C.c_void_p * n)(*([SENTINEL] * n))
    st = lib.peps_env_boundary(sess.ctx.handle, arr, n, C.byref(opts), out)
    handles = [out[i] for i in range(n)]
    if st == 0:
        for h in handles:
            lib.peps_env_free(h)
    return st, handles, lib.peps_last_error().decode()


def raw_state(tensors, shapes=None):
    st = binding.state_of(tensors)
    if shapes is not None:   # declared dimensions that differ from the tensors'
        flat = [int(x) for row in shapes for s in row for x in s]
        st.dims = (C.c_int32 * len(flat))(*flat)
        st.shapes = shapes
    return st


def opts(chi=4, **kw):
    o = binding.Context.opts(chi)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


INVALID, OOM, NOT_CONVERGED, NONFINITE = -1, -2, -4, -5


def test_invalid_requests_leave_outputs_null(sess):
    say("invalid requests")
    A = binding.to_device(make_peps(3, 3, 2, "uniform", 5))
    shapes = [[tuple(t.shape) for t in row] for row in A]
    cases = []
    bad = [list(map(list, row)) for row in shapes]
    bad[0][0][1] = 2                                   # left edge leg of dimension 2
    cases.append(("edge leg", raw_state(A, [[tuple(s) for s in row] for row in bad]), opts()))
    bad = [list(map(list, row)) for row in shapes]
    bad[1][1][3] = 3                                   # right leg differs from its neighbour's left leg
    cases.append(("bond mismatch", raw_state(A, [[tuple(s) for s in row] for row in bad]), opts()))
    cases.append(("chi 0", raw_state(A), opts(chi=0)))
    cases.append(("dtype", raw_state(A), opts(dtype=7)))
    cases.append(("reserved", raw_state(A), opts(reserved=1)))
    cases.append(("tol", raw_state(A), opts(tol=1.5)))
    cases.append(("cap below minimum", raw_state(A), opts(tol=1e-12, halfsweeps=6, max_halfsweeps=4)))
    cases.append(("unknown flag", raw_state(A), opts(flags=64)))
    for name, st, o in cases:
        code, out, msg = call_boundary(sess, [st], o)
        assert code == INVALID, (name, code, msg)
        assert out == [None], name
        assert msg, name


def test_window_out_of_range(sess):
    say("window out of range")
    lib = sess.ctx.lib
    A = binding.to_device(make_peps(4, 4, 2, "uniform", 6))
    st = raw_state(A)
    arr = (binding.State * 1)(st.struct())
    for w in [(0, 0, 4, 0, 1, 0, 0), (0, 1, 2, 0, 1, 0, 0), (1, 0, 1, 0, 1, 0, 0), (0, 0, 1, 2, 1, 0, 2)]:
        win = (binding.Window * 1)(binding.Window(*w))
        out = (C.c_void_p * 1)(SENTINEL)
        o = opts()
        code = lib.peps_cluster_env(sess.ctx.handle, arr, 1, win, 1, C.byref(o), out)
        assert code == INVALID, (w, code)
        assert out[0] is None, w


def test_nonfinite_input_is_rejected_before_compute(sess):
    import torch
    say("non-finite input")
    A = binding.to_device(make_peps(3, 4, 2, "normal_unit", 7))
    for bad, val in (((1, 2), float("nan")), ((2, 3), float("inf"))):
        B = [[t.clone() for t in row] for row in A]
        B[bad[0]][bad[1]].view(-1)[3] = val
        code, out, msg = call_boundary(sess, [raw_state(B)], opts())
        assert code == NONFINITE, (bad, code, msg)
        assert out == [None]
        assert f"site ({bad[0]},{bad[1]})" in msg, msg
    # the same check guards the cluster entry point
    B = [[t.clone() for t in row] for row in A]
    B[0][1].view(-1)[0] = float("nan")
    st = raw_state(B)
    arr = (binding.State * 1)(st.struct())
    win = (binding.Window * 1)(binding.Window(0, 0, 1, 0, 1, 0, 0))
    out = (C.c_void_p * 1)(SENTINEL)
    o = opts()
    assert sess.ctx.lib.peps_cluster_env(sess.ctx.handle, arr, 1, win, 1, C.byref(o), out) == NONFINITE
    assert out[0] is None
    torch.cuda.synchronize()


def test_workspace_cap_below_one_sandwich_is_oom(sess):
    say("workspace cap")
    ctx = binding.Context(0, sess.stream.cuda_stream)
    A = binding.to_device(make_peps(6, 6, 4, "near_product", 8))
    env = ctx.env_boundary_raw([binding.state_of(A)], 32)[0]
    ctx.set_workspace(1 << 20)
    with pytest.raises(binding.PepsError) as ei:
        ctx.expect([env])
    assert ei.value.code == OOM
    ctx.set_workspace(48 << 30)
    r = ctx.expect([env])[0]   # the environment is still usable
    assert np.all(np.isfinite(r["bond_h"]))
    env.free()
    ctx.close()


def test_not_converged_flag_and_strict(sess):
    """A row that reaches the cap before the tolerance is counted by
    peps_env_info; with PEPS_OPTS_STRICT the call fails instead."""
    say("not converged")
    A = make_peps(5, 5, 2, "uniform", 9)
    dev = binding.to_device(A)
    env = sess.env_boundary([dev], 3, halfsweeps=2, tol=1e-12, max_halfsweeps=60)[0]
    w, sweeps, unconv = env.info(full=True)
    env.free()
    assert unconv >= 1 and np.max(sweeps) == 60
    o = opts(chi=3, halfsweeps=2, tol=1e-12, max_halfsweeps=60, flags=binding.OPTS_STRICT)
    code, out, msg = call_boundary(sess, [raw_state(dev)], o)
    assert code == NOT_CONVERGED and out == [None], (code, msg)

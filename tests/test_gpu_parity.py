"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Float64 results must agree with the oracle to 1e-10 (absolute on <S^z> and
bond energies, which are O(1) bounded quantities, and on log <psi|psi>);
the oracle runs the same algorithm (same caps, same SplitMix64 start, same
half-sweeps), so the two differ only by rounding order.
"""
import sys

import numpy as np
import pytest

from oracle import api, exact
from paper_1311_6696_amd import binding
from paper_1311_6696_amd.inputs import make_peps, product_state, workload_peps, WORKLOADS

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sess():
    return binding.Session(0)


def run_gpu(sess, A_list, chi, dtype="f64", H=4):
    dev = [binding.to_device(A) for A in A_list]
    envs = sess.env_boundary(dev, chi, dtype, H)
    res = sess.expect(envs)
    info = [e.info() for e in envs]
    for e in envs:
        e.free()
    return res, info


def max_obs_diff(r, ref):
    out = 0.0
    for k in ("sz", "bond_h", "bond_v"):
        if np.asarray(ref[k]).size:
            out = max(out, float(np.max(np.abs(np.asarray(r[k]) - np.asarray(ref[k])))))
    return out


@pytest.mark.parametrize("seed", [1001, 1002, 1003])
def test_4x4_D2_exact_vs_statevector(sess, seed):
    say(f"4x4 D=2 chi=16 seed={seed}")
    A = make_peps(4, 4, 2, "uniform", seed)
    (r,), _ = run_gpu(sess, [A], 16)
    sv = exact.sv_observables(A)
    ref = api.expect(api.env_boundary(A, 16))
    assert max_obs_diff(r, ref) < TOL64
    assert max_obs_diff(r, sv) < TOL64
    assert abs(r["log_norm"] - np.log(sv["norm"])) < TOL64
    assert r["sign"] == 1.0


@pytest.mark.parametrize("case", [
    (3, 4, 2, "normal_unit", 4, 4),
    (4, 3, 3, "normal_unit", 5, 3),
    (5, 5, 2, "near_product", 6, 4),
    (1, 5, 2, "uniform", 4, 2),
    (5, 1, 2, "uniform", 4, 2),
    (4, 4, 3, "uniform", 9, 1),
])
def test_truncated_parity(sess, case):
    Lr, Lc, D, dist, chi, H = case
    say(f"truncated {case}")
    A = make_peps(Lr, Lc, D, dist, 100 + Lr * 10 + Lc)
    (r,), (info,) = run_gpu(sess, [A], chi, H=H)
    env = api.env_boundary(A, chi, H)
    ref = api.expect(env)
    assert max_obs_diff(r, ref) < TOL64
    assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))
    # ALS diagnostics: squared centre norms per half-sweep agree with the oracle's
    om = [i.omegas for row in (env.top, env.bottom) for (_, _, i) in row[1:] if i is not None and not i.exact]
    if om:
        got = np.sort(info.reshape(-1))
        want = np.sort(np.array(om).reshape(-1))
        np.testing.assert_allclose(got, want, rtol=1e-10)


def test_tolerance_stop_parity(sess):
    """ALS with the omega tolerance: every truncated row runs the oracle's
    number of half-sweeps (on this state no stopping decision lies within
    10 % of the tolerance, so rounding cannot flip one), with the same
    squared centre norms, and the observables agree."""
    say("tolerance stop 4x4 D=3 chi=6")
    A = make_peps(4, 4, 3, "near_product", 8)
    env = sess.env_boundary([binding.to_device(A)], 6, halfsweeps=2, tol=1e-12, max_halfsweeps=60)[0]
    r = sess.expect([env])[0]
    w, sweeps, unconv = env.info(full=True)
    env.free()
    oenv = api.env_boundary(A, 6, 2, tol=1e-12, max_halfsweeps=60)
    ref = api.expect(oenv)
    rows = [i for row in (oenv.top, oenv.bottom) for (_, _, i) in row[1:] if not i.exact]
    assert unconv == 0
    assert list(sweeps) == [len(i.omegas) for i in rows]
    for k, i in enumerate(rows):
        np.testing.assert_allclose(w[k, :len(i.omegas)], i.omegas, rtol=1e-10)
        assert np.all(np.isnan(w[k, len(i.omegas):]))
    assert max_obs_diff(r, ref) < TOL64
    assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))


def test_10x10_D6_chi72_top_boundaries_vs_oracle(sess):
    """The precision workload's own shape (10x10, D=6, chi=72, FP64): the
    top boundaries after rows 0, 1 and 2 against the oracle's (2592 x 72 QR
    blocks, unfused D=6 chain stages): squared centre norms per half-sweep
    to 1e-10, every tensor to 1e-8 of its largest entry (the QR gauge with
    R_ii >= 0 fixes them), boundary fidelity 1 - f <= 1e-12 and the log-scale
    to 1e-10.  The oracle part takes about half a minute of host time."""
    from oracle import boundary
    from oracle.boundary import whole_lattice
    say("10x10 D=6 chi=72 rows 0-2 vs oracle")
    A = workload_peps("10x10_D6_chi72")
    env = sess.env_boundary([binding.to_device(A)], 72)[0]
    info = env.info()
    lat = whole_lattice(A)
    T, s = boundary.trivial_boundary(lat.tau), 0.0
    for r in range(3):
        T, dl, oinfo = boundary.absorb_row(T, lat.A[r], lat.lam[r], lat.rho[r], 72, 4, api.DEFAULT_SEED, 0, r)
        s += dl
        X, ls = env.mps(0, r + 1)
        X = [x.cpu().numpy() for x in X]
        assert abs(ls - s) < TOL64 * max(1.0, abs(s)), r
        for x, t in zip(X, T):
            assert x.shape == t.shape
            assert np.abs(x - t).max() <= 1e-8 * np.abs(t).max(), r
        assert 1.0 - boundary.boundary_fidelity(X, T) <= 1e-12, r
        if not oinfo.exact:
            np.testing.assert_allclose(info[r - 1, :4], oinfo.omegas, rtol=1e-10)
    env.free()


def test_3x3_D8_chi64_full_environment_vs_oracle(sess):
    """D = 8 (the largest bond of the batched-instances draw) at chi = D^2 =
    64: the whole environment of a 3x3 U[0,1) lattice (one truncated row per
    side, D=8 two-row sandwiches) against the oracle, about a minute of host
    time."""
    say("3x3 D=8 chi=64 vs oracle")
    A = make_peps(3, 3, 8, "uniform", 1008)
    (r,), _ = run_gpu(sess, [A], 64)
    ref = api.expect(api.env_boundary(A, 64))
    assert max_obs_diff(r, ref) < TOL64
    assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))


def test_product_state(sess):
    say("product state 3x5")
    A = product_state(3, 5, seed=2)
    (r,), _ = run_gpu(sess, [A], 3)
    ref = api.expect(api.env_boundary(A, 3))
    assert max_obs_diff(r, ref) < 1e-13


def test_batched_heterogeneous(sess):
    """Lattices of different shapes in one call give the single-call results."""
    say("batched heterogeneous")
    As = [make_peps(3, 4, 2, "normal_unit", 21), make_peps(4, 3, 3, "uniform", 22),
          make_peps(5, 5, 2, "near_product", 23)]
    res, _ = run_gpu(sess, As, 5, H=3)
    for A, r in zip(As, res):
        ref = api.expect(api.env_boundary(A, 5, 3))
        assert max_obs_diff(r, ref) < TOL64


def test_batched_large_launches_match_single_lattices(sess):
    """Eight 8x8 D=4 chi=32 lattices in one call: the chain-step launches are
    large enough for each workgroup to make several x passes and the column
    steps run without x slices, unlike one lattice per call; every lattice's
    observables and log-norm agree with its own single-lattice run (whose
    parity with the oracle is checked at full size elsewhere)."""
    say("8 x (8x8 D=4 chi=32) batched against single")
    As = [make_peps(8, 8, 4, "near_product", 3000 + i) for i in range(8)]
    batch, _ = run_gpu(sess, As, 32)
    for A, rb in zip(As, batch):
        (rs,), _ = run_gpu(sess, [A], 32)
        # (different launch shapes sum in different orders: rounding differences only)
        assert max_obs_diff(rb, rs) < TOL64
        assert abs(rb["log_norm"] - rs["log_norm"]) < TOL64 * max(1.0, abs(rs["log_norm"]))


def test_batched_per_state_chi(sess):
    """Instances of different L, D and chi = D^2 (the batched-instances
    recipe at small sizes) in one call, one options record per state."""
    say("batched per-state chi")
    pairs = [(4, 2), (5, 3), (3, 3), (6, 2)]
    As = [make_peps(L, L, D, "uniform", 40 + k) for k, (L, D) in enumerate(pairs)]
    chis = [D * D for (_, D) in pairs]
    envs = sess.env_boundary([binding.to_device(A) for A in As], chis, "f64", 3)
    res = sess.expect(envs)
    for e in envs:
        e.free()
    for A, chi, r in zip(As, chis, res):
        ref = api.expect(api.env_boundary(A, chi, 3))
        assert max_obs_diff(r, ref) < TOL64
        assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))


def test_batched_per_state_seed_and_halfsweeps(sess):
    """Per-state records with different chi, half-sweep counts and seeds in
    one precision: each state keeps its own ALS start and sweep count."""
    say("batched per-state chi/halfsweeps/seed")
    As = [make_peps(4, 4, 2, "normal_unit", 21), make_peps(5, 4, 2, "uniform", 22),
          make_peps(4, 5, 3, "normal_unit", 23)]
    chis, Hs, seeds = [4, 3, 6], [3, 5, 4], [11, 12, 13]
    envs = sess.env_boundary([binding.to_device(A) for A in As], chis, "f64", Hs, seeds)
    res = sess.expect(envs)
    for e in envs:
        e.free()
    for A, r, chi, H, seed in zip(As, res, chis, Hs, seeds):
        ref = api.expect(api.env_boundary(A, chi, H, seed))
        assert max_obs_diff(r, ref) < TOL64


# --- vertical bonds from the left/right boundaries (column sandwiches) -------

def _aniso_peps(Lr, Lc, Dh, Dv, seed):
    rng = np.random.default_rng(seed)
    return [[rng.standard_normal((2, 1 if c == 0 else Dh, 1 if r == 0 else Dv,
                                  1 if c == Lc - 1 else Dh, 1 if r == Lr - 1 else Dv))
             for c in range(Lc)] for r in range(Lr)]


def run_cols(sess, A_list, chi, dtype="f64", H=4):
    envs = sess.env_boundary([binding.to_device(A) for A in A_list], chi, dtype, H, columns=True)
    res = sess.expect(envs)
    for e in envs:
        e.free()
    return res


@pytest.mark.parametrize("case", [
    ("normal_unit", 3, 4, 2, 4096, 4),   # lossless chi
    ("normal_unit", 3, 4, 2, 4, 4),
    ("normal_unit", 4, 3, 3, 5, 3),
    ("aniso", 3, 4, 0, 6, 4),            # horizontal bonds 2, vertical bonds 3
    ("near_product", 5, 5, 2, 4, 4),
    ("uniform", 1, 5, 2, 4, 2),
    ("uniform", 5, 1, 2, 4, 2),
])
def test_columns_parity(sess, case):
    dist, Lr, Lc, D, chi, H = case
    say(f"columns {case}")
    A = (_aniso_peps(Lr, Lc, 2, 3, 90 + Lr * Lc) if dist == "aniso"
         else make_peps(Lr, Lc, D, dist, 200 + Lr * 10 + Lc))
    (r,) = run_cols(sess, [A], chi, H=H)
    ref = api.expect(api.env_boundary(A, chi, H), columns=api.env_columns(A, chi, H))
    assert max_obs_diff(r, ref) < TOL64
    assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))
    if chi == 4096:
        assert max_obs_diff(r, exact.sv_observables(A)) < TOL64


def test_columns_mixed_with_row_only_envs(sess):
    """Environments with and without column boundaries in one expect call."""
    say("columns mixed with two-row environments")
    A1, A2 = make_peps(4, 5, 2, "normal_unit", 301), make_peps(5, 4, 2, "uniform", 302)
    e1 = sess.env_boundary([binding.to_device(A1)], 4, "f64", 3, columns=True)
    e2 = sess.env_boundary([binding.to_device(A2)], 4, "f64", 3)
    r1, r2 = sess.expect(e1 + e2)
    for e in e1 + e2:
        e.free()
    assert max_obs_diff(r1, api.expect(api.env_boundary(A1, 4, 3), columns=api.env_columns(A1, 4, 3))) < TOL64
    assert max_obs_diff(r2, api.expect(api.env_boundary(A2, 4, 3))) < TOL64


def test_columns_for_cluster_windows(sess):
    """Cluster windows with column boundaries: the bond downwards from the
    single-column sandwich of the transposed window, against the oracle."""
    from oracle import cluster
    from oracle.boundary import whole_lattice
    say("columns in cluster windows")
    L, n, chi = 5, 3, 4
    A = make_peps(L, L, 2, "near_product", 501)
    wins = []
    for (i, j) in [(0, 0), (2, 2), (3, 1), (1, 4)]:
        r0, r1 = cluster.window_bounds(i, n, L)
        c0, c1 = cluster.window_bounds(j, n, L)
        wins.append((0, r0, r1, c0, c1, i, j))
    dev = binding.to_device(A)
    st = binding.state_of(dev)
    ctx = sess.ctx
    import ctypes as C
    o = ctx.opts(chi)
    o.flags = binding.OPTS_COLUMNS
    arr = (binding.State * 1)(st.struct())
    w = (binding.Window * len(wins))(*[binding.Window(*x) for x in wins])
    out = (C.c_void_p * len(wins))()
    binding._check(ctx.lib, ctx.lib.peps_cluster_env(ctx.handle, arr, 1, w, len(wins), C.byref(o), out))
    envs = [binding.Env(ctx, out[k], x[2] - x[1] + 1, x[4] - x[3] + 1, window=True) for k, x in enumerate(wins)]
    res = sess.expect(envs)
    for e in envs:
        e.free()
    sep = cluster.SeparableEnv(whole_lattice(A))
    for x, r in zip(wins, res):
        _, r0, r1, c0, c1, i, j = x
        win = cluster.window_lattice(sep, r0, r1, c0, c1)
        ref = api.expect(api.env_boundary(win, chi), rows=[i - r0], columns=api.env_columns(win, chi))
        assert abs(r["sz"] - ref["sz"][i - r0, j - c0]) < TOL64
        if j < c1:
            assert abs(r["right"] - ref["bond_h"][i - r0, j - c0]) < TOL64
        if i < r1:
            assert abs(r["down"] - ref["bond_v"][i - r0, j - c0]) < TOL64
        else:
            assert np.isnan(r["down"])


# --- boundary overlaps (boundary fidelity) -------------------------------------

def test_boundary_overlap_parity(sess):
    """<X|Y>, <X|X>, <Y|Y> of stored boundaries from all four sides, between
    a lossless and a truncated environment (different seeds), against the
    oracle; lossless boundaries from two seeds have fidelity 1."""
    say("boundary overlaps")
    A = make_peps(5, 4, 2, "normal_unit", 401)
    dev = binding.to_device(A)
    ea = sess.env_boundary([dev], 1024, "f64", 4, 1, columns=True)[0]
    ea2 = sess.env_boundary([dev], 1024, "f64", 4, 2, columns=True)[0]
    eb = sess.env_boundary([dev], 3, "f64", 4, 2, columns=True)[0]
    reqs = [(ea, x, s, k) for x in (ea2, eb) for s in range(4) for k in range(1, 5 if s < 2 else 4)]
    res = sess.ctx.boundary_overlap(reqs)
    for e in (ea, ea2, eb):
        e.free()
    ref = {1024: (api.env_boundary(A, 1024, 4, 1), api.env_columns(A, 1024, 4, 1)),
           3: (api.env_boundary(A, 3, 4, 2), api.env_columns(A, 3, 4, 2))}
    for (a, x, s, k), (xy, xx, yy) in zip(reqs, res):
        f = abs(xy) / np.sqrt(xx * yy)
        if x is ea2:
            assert abs(1.0 - f) < 1e-12
            continue
        ra, rb = (ref[1024][0], ref[3][0]) if s < 2 else (ref[1024][1], ref[3][1])
        assert abs(f - api.boundary_fidelity(ra, rb, s % 2, k)) < TOL64
        assert abs(xx - 1.0) < 1e-12 and abs(yy - 1.0) < 1e-12


def test_boundary_overlap_rejects_bad_requests(sess):
    A = make_peps(3, 3, 2, "uniform", 5)
    e = sess.env_boundary([binding.to_device(A)], 4)[0]
    with pytest.raises(binding.PepsError):   # no column boundaries
        sess.ctx.boundary_overlap([(e, e, 2, 1)])
    with pytest.raises(binding.PepsError):   # k out of range
        sess.ctx.boundary_overlap([(e, e, 0, 3)])
    with pytest.raises(binding.PepsError):   # closing boundary
        sess.ctx.boundary_overlap([(e, e, 1, 0)])
    e.free()


@pytest.mark.parametrize("L,D,chi,dist,seed", [
    (4, 3, 72, "normal_unit", 61),   # 81 x 72 QR blocks: five columns per wave
    (4, 5, 30, "uniform", 52),       # 625 x 30 and 625 x 25 blocks: tree QR over row blocks
])
def test_wide_and_tall_qr_blocks(sess, L, D, chi, dist, seed):
    """Truncated rows whose QR blocks need the widest register variant or the
    row-block tree (TSQR) give the oracle's results."""
    say(f"qr blocks L={L} D={D} chi={chi}")
    A = make_peps(L, L, D, dist, seed)
    (r,), _ = run_gpu(sess, [A], chi, H=2)
    ref = api.expect(api.env_boundary(A, chi, 2))
    assert max_obs_diff(r, ref) < TOL64
    assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))


def test_graph_replay_bitwise(sess):
    """Launch sequences replayed from captured HIP graphs give the op-by-op
    results bit for bit, also after new tensor values are written into the
    same device buffers (the replay reads them at execution time)."""
    say("graph replay")
    A1 = make_peps(5, 5, 3, "normal_unit", 71)
    A2 = make_peps(5, 5, 3, "normal_unit", 72)
    dev = binding.to_device(A1)

    def one():
        envs = sess.env_boundary([dev], 7, "f64", 3)
        r = sess.expect(envs)[0]
        for e in envs:
            e.free()
        return r

    def load(A):
        for row_d, row_h in zip(dev, A):
            for t, h in zip(row_d, row_h):
                t.copy_(binding.to_device([[h]])[0][0])

    plain1 = one()
    load(A2)
    plain2 = one()
    load(A1)
    sess.ctx.graphs(True)
    try:
        replay = [one(), one()]   # capture, then replay
        load(A2)
        replay2 = one()
    finally:
        sess.ctx.graphs(False)
    for r in replay:
        for k in ("sz", "bond_h", "bond_v"):
            assert np.array_equal(r[k], plain1[k])
        assert r["log_norm"] == plain1["log_norm"]
    for k in ("sz", "bond_h", "bond_v"):
        assert np.array_equal(replay2[k], plain2[k])
    ref = api.expect(api.env_boundary(A2, 7, 3))
    assert max_obs_diff(replay2, ref) < TOL64


def test_autotuned_shapes(sess):
    """Launch shapes chosen by timing give the oracle's results, while tuning
    and afterwards from the stored choices."""
    say("autotune")
    A = make_peps(6, 6, 3, "normal_unit", 81)
    ref = api.expect(api.env_boundary(A, 9, 3))
    sess.ctx.autotune(1)
    try:
        (r1,), _ = run_gpu(sess, [A], 9, H=3)
    finally:
        sess.ctx.autotune(0)
    (r2,), _ = run_gpu(sess, [A], 9, H=3)
    sess.ctx.autotune(2)
    for r in (r1, r2):
        assert max_obs_diff(r, ref) < TOL64
        assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))


def test_8x8_D4_chi32_full_parity(sess):
    """8x8, D=4, near-product, chi=32: all 112 bonds and the norm."""
    say("8x8 D=4 chi=32 f64")
    c = WORKLOADS["8x8_D4_chi32"]
    A = workload_peps("8x8_D4_chi32")
    (r,), _ = run_gpu(sess, [A], c["chi"])
    ref = api.expect(api.env_boundary(A, c["chi"]))
    assert max_obs_diff(r, ref) < TOL64
    assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))


def test_8x8_D4_chi32_columns_full_parity(sess):
    """8x8, D=4, near-product, chi=32 with column boundaries: all 112 bonds
    (vertical ones from the column sandwiches) and the norm."""
    say("8x8 D=4 chi=32 f64 columns")
    c = WORKLOADS["8x8_D4_chi32"]
    A = workload_peps("8x8_D4_chi32")
    (r,) = run_cols(sess, [A], c["chi"])
    ref = api.expect(api.env_boundary(A, c["chi"]), columns=api.env_columns(A, c["chi"]))
    assert max_obs_diff(r, ref) < TOL64
    assert abs(r["log_norm"] - ref["log_norm"]) < TOL64 * max(1.0, abs(ref["log_norm"]))


def test_10x10_D6_chi72_properties(sess):
    """10x10, D=6, N(0,1) unit-norm sites, chi=72 (the precision workload's
    size, too large for the oracle): properties that hold at any size.
    Bounds of <S^z> and <S.S>; the site environments reproduce <S^z> of the
    row sandwich (A N A = sign, (S^z A) N A = <S^z> sign); FP32 agrees with
    FP64; boundaries have unit norm and the FP32 ones fidelity ~1."""
    from oracle import spin
    say("10x10 D=6 chi=72 properties")
    A = workload_peps("10x10_D6_chi72")
    c = WORKLOADS["10x10_D6_chi72"]
    dev = binding.to_device(A)
    e64 = sess.env_boundary([dev], c["chi"], "f64", 4)[0]
    e32 = sess.env_boundary([dev], c["chi"], "f32", 4)[0]
    r64, = sess.expect([e64])
    r32, = sess.expect([e32])
    assert np.all(np.abs(r64["sz"]) <= 0.5 + 1e-9)
    for k in ("bond_h", "bond_v"):
        assert np.all(r64[k] >= -0.75 - 1e-9) and np.all(r64[k] <= 0.25 + 1e-9)
        assert np.abs(r32[k] - r64[k]).max() < 1e-4
    sites = [(0, 0), (0, 5), (4, 4), (9, 9)]
    got, _ = sess.site_env([(e64, r, q) for r, q in sites])
    for (r, q), (N, _, sign) in zip(sites, got):
        N = N.cpu().numpy()
        a = A[r][q].reshape(2, -1)
        sa = sandwich_apply(spin.SZ, A[r][q]).reshape(2, -1)
        assert abs(np.einsum("pk,kj,pj->", a, N, a) - sign) < 1e-9
        assert abs(np.einsum("pk,kj,pj->", sa, N, a) * sign - r64["sz"][r, q]) < 1e-9
    ov = sess.ctx.boundary_overlap([(e64, e32, side, k) for side in (0, 1) for k in (1, 5, 9)])
    for xy, xx, yy in ov:
        assert abs(xx - 1.0) < 1e-10
        assert 1.0 - abs(xy) / np.sqrt(xx * yy) < 1e-6
    e64.free()
    e32.free()


def sandwich_apply(O, A):
    """O on the physical leg of a site tensor (the operator convention of the
    sandwich: sum_q O[p, q] A[q, ...])."""
    return np.tensordot(O, A, axes=([1], [0]))


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-6), ("bf16", 5e-3)])
def test_precision_forms_error(sess, dtype, tol):
    """FP32 / BF16 bulk contractions (FP64 QR and norms): relative energy
    error against the FP64 oracle within the stated bound (measured on this
    6x6 D=3 chi=9 state: FP32 7e-8, BF16 2.6e-3, whose operands keep 8
    significant bits)."""
    say(f"precision form {dtype}")
    A = make_peps(6, 6, 3, "normal_unit", 31)
    (r,), _ = run_gpu(sess, [A], 9, dtype=dtype)
    ref = api.expect(api.env_boundary(A, 9))
    e_ref = api.energy(ref)
    e = float(np.sum(r["bond_h"]) + np.sum(r["bond_v"]))
    err = abs(e - e_ref) / abs(e_ref)
    say(f"  {dtype}: relative energy error {err:.3e}, max bond error {max_obs_diff(r, ref):.3e}")
    assert err < tol

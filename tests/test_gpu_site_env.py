"""Norm environments N_l of single sites and right-hand sides b_l of gated
bonds (the two sides of the ALS tensor update) on the GPU, through the C
ABI, against the FP64 oracle: whole lattices, cluster windows, batching, the
full 8x8 D=4 chi=32 workload and the FP32 form."""
import sys

import numpy as np
import pytest

from oracle import api, cluster
from oracle.boundary import whole_lattice
from paper_1311_6696_amd import binding
from paper_1311_6696_amd.inputs import make_peps, workload_peps, WORKLOADS

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sess():
    return binding.Session(0)


def check(got, ref, tol):
    (N, lz, sg), (Nr, lzr, sgr) = got, ref
    N = N.cpu().numpy()
    assert N.shape == Nr.shape
    assert np.abs(N - Nr).max() <= tol * max(1.0, np.abs(Nr).max())
    assert abs(lz - lzr) <= tol * max(1.0, abs(lzr))
    assert sg == sgr


@pytest.mark.parametrize("case", [
    (3, 4, 2, "normal_unit", 4096, 4),   # lossless chi
    (4, 3, 3, "normal_unit", 5, 3),
    (5, 5, 2, "near_product", 4, 4),
    (1, 4, 2, "uniform", 4, 2),
    (4, 1, 2, "uniform", 4, 2),
])
def test_site_env_parity_every_site(sess, case):
    Lr, Lc, D, dist, chi, H = case
    say(f"site environments {case}")
    A = make_peps(Lr, Lc, D, dist, 300 + Lr * 10 + Lc)
    env = sess.env_boundary([binding.to_device(A)], chi, "f64", H)[0]
    sites = [(r, c) for r in range(Lr) for c in range(Lc)]
    got, fl = sess.site_env([(env, r, c) for r, c in sites])
    env.free()
    ref_env = api.env_boundary(A, chi, H)
    for (r, c), g in zip(sites, got):
        check(g, api.site_env(ref_env, r, c), TOL64)
    assert fl > 0


def test_site_env_batched_over_lattices(sess):
    """Requests on two lattices of different shapes in one call."""
    say("site environments batched over two lattices")
    A1, A2 = make_peps(4, 5, 2, "normal_unit", 311), make_peps(5, 3, 3, "uniform", 312)
    e1, e2 = sess.env_boundary([binding.to_device(A1), binding.to_device(A2)], [4, 6], "f64", 3)
    reqs = [(e1, 0, 0), (e2, 4, 2), (e1, 2, 3), (e2, 1, 1), (e1, 2, 1)]
    got, _ = sess.site_env(reqs)
    r1, r2 = api.env_boundary(A1, 4, 3), api.env_boundary(A2, 6, 3)
    for (e, r, c), g in zip(reqs, got):
        check(g, api.site_env(r1 if e is e1 else r2, r, c), TOL64)
    # the environments still give their observables afterwards
    res = sess.expect([e1])[0]
    assert np.abs(res["sz"] - api.expect(r1)["sz"]).max() < TOL64
    e1.free()
    e2.free()


def test_site_env_of_cluster_windows(sess):
    """Centre-site environments of n = 3 windows (cut legs closed by CU_0):
    the environment a cluster update of that site uses."""
    say("site environments of n=3 windows")
    L, n, chi = 5, 3, 4
    A = make_peps(L, L, 2, "near_product", 321)
    sample = [(0, 0), (2, 2), (4, 1), (1, 4)]
    wins = []
    for (i, j) in sample:
        r0, r1 = cluster.window_bounds(i, n, L)
        c0, c1 = cluster.window_bounds(j, n, L)
        wins.append((0, r0, r1, c0, c1, i, j))
    envs = sess.cluster_env([binding.to_device(A)], wins, chi, "f64", 4)
    got, _ = sess.site_env([(e, w[5] - w[1], w[6] - w[3]) for e, w in zip(envs, wins)])
    for e in envs:
        e.free()
    sep = cluster.SeparableEnv(whole_lattice(A))
    for w, g in zip(wins, got):
        _, r0, r1, c0, c1, i, j = w
        wenv = api.env_boundary(cluster.window_lattice(sep, r0, r1, c0, c1), chi, 4)
        check(g, api.site_env(wenv, i - r0, j - c0), TOL64)


def test_site_env_8x8_D4_chi32_sample(sess):
    """8x8, D=4, near-product, chi=32: every site in one batched call, a
    sample (corner, edges, bulk) against the oracle."""
    say("site environments 8x8 D=4 chi=32")
    c = WORKLOADS["8x8_D4_chi32"]
    A = workload_peps("8x8_D4_chi32")
    env = sess.env_boundary([binding.to_device(A)], c["chi"], "f64", 4)[0]
    sites = [(r, s) for r in range(8) for s in range(8)]
    got, _ = sess.site_env([(env, r, s) for r, s in sites])
    env.free()
    ref_env = api.env_boundary(A, c["chi"], 4)
    for k in (0, 7, 19, 27, 36, 56, 63):
        r, s = sites[k]
        check(got[k], api.site_env(ref_env, r, s), TOL64)


def test_site_env_fp32_form(sess):
    """FP32 contractions (FP64 QR and norms): error against the FP64 oracle."""
    say("site environments fp32")
    A = make_peps(5, 5, 3, "normal_unit", 331)
    env = sess.env_boundary([binding.to_device(A)], 9, "f32", 4)[0]
    sites = [(0, 0), (2, 2), (4, 3)]
    got, _ = sess.site_env([(env, r, c) for r, c in sites])
    env.free()
    ref_env = api.env_boundary(A, 9, 4)
    for (r, c), g in zip(sites, got):
        check(g, api.site_env(ref_env, r, c), 1e-4)


def test_site_env_rejects_bad_requests(sess):
    A = make_peps(3, 3, 2, "uniform", 5)
    env = sess.env_boundary([binding.to_device(A)], 4)[0]
    with pytest.raises(binding.PepsError):
        sess.ctx.site_env_raw([(env, 3, 0, 1 << 20)])
    with pytest.raises(binding.PepsError):
        sess.ctx.site_env_raw([(env, 0, 0, 0)])
    env.free()


def test_strip_cluster_site_env(sess):
    """A strip cluster (delta = 3 rows around row 2, every column) is a
    window spanning the lattice's width: its boundaries, observables and the
    environments of the centre row's sites for a strip cluster update."""
    say("strip cluster delta=3")
    L, chi = 6, 4
    A = make_peps(L, L, 2, "near_product", 341)
    wins = [(0, 1, 3, 0, L - 1, 2, j) for j in range(L)]
    envs = sess.cluster_env([binding.to_device(A)], wins, chi, "f64", 4)
    res = sess.expect(envs)
    got, _ = sess.site_env([(e, 1, w[6]) for e, w in zip(envs, wins)])
    for e in envs:
        e.free()
    sep = cluster.SeparableEnv(whole_lattice(A))
    wenv = api.env_boundary(cluster.window_lattice(sep, 1, 3, 0, L - 1), chi, 4)
    ref = api.expect(wenv, rows=[1])
    for w, r, g in zip(wins, res, got):
        j = w[6]
        assert abs(r["sz"] - ref["sz"][1, j]) < TOL64
        if j < L - 1:
            assert abs(r["right"] - ref["bond_h"][1, j]) < TOL64
        check(g, api.site_env(wenv, 1, j), TOL64)


def test_site_env_with_column_environment_and_fp32_columns(sess):
    """Site environments of an environment that also holds column
    boundaries; the column path in the FP32 form against the FP64 oracle."""
    say("site env on a column environment; fp32 columns")
    A = make_peps(4, 5, 2, "normal_unit", 351)
    env = sess.env_boundary([binding.to_device(A)], 4, "f64", 4, columns=True)[0]
    got, _ = sess.site_env([(env, 1, 3), (env, 3, 0)])
    env.free()
    ref_env = api.env_boundary(A, 4, 4)
    check(got[0], api.site_env(ref_env, 1, 3), TOL64)
    check(got[1], api.site_env(ref_env, 3, 0), TOL64)
    env32 = sess.env_boundary([binding.to_device(A)], 4, "f32", 4, columns=True)[0]
    r = sess.expect([env32])[0]
    env32.free()
    ref = api.expect(ref_env, columns=api.env_columns(A, 4, 4))
    for k in ("sz", "bond_h", "bond_v"):
        assert np.abs(r[k] - ref[k]).max() < 1e-5


# --- right-hand sides b_l of a gated horizontal bond -------------------------

def _gate(seed):
    return np.random.default_rng(seed).standard_normal((2, 2, 2, 2))


def _heisenberg_gate(tau):
    """exp(-tau S.S) on two spins 1/2, G[p, P, q, Q]."""
    from oracle import spin
    h = sum(w * np.kron(a, b) for w, a, b in spin.BOND_TERMS)
    ev, U = np.linalg.eigh(h)
    return (U @ np.diag(np.exp(-tau * ev)) @ U.T).reshape(2, 2, 2, 2)


def _dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def check_b(got, ref, tol):
    for g, r in zip(got, ref):
        g = g.cpu().numpy()
        assert g.shape == r.shape
        assert np.abs(g - r).max() <= tol * max(1.0, np.abs(r).max())


@pytest.mark.parametrize("case", [
    ("normal_unit", 3, 4, 4096, 4),   # lossless chi
    ("normal_unit", 4, 4, 3, 4),
    ("aniso", 3, 4, 5, 3),
    ("uniform", 1, 4, 4, 2),
])
def test_bond_env_parity_every_bond(sess, case):
    dist, Lr, Lc, chi, H = case
    say(f"bond environments {case}")
    if dist == "aniso":
        rng = np.random.default_rng(360)
        A = [[rng.standard_normal((2, 1 if c == 0 else 2, 1 if r == 0 else 3, 1 if c == Lc - 1 else 2,
                                   1 if r == Lr - 1 else 3)) for c in range(Lc)] for r in range(Lr)]
    else:
        A = make_peps(Lr, Lc, 2, dist, 361 + Lr * Lc)
    G = _gate(Lr * Lc)
    env = sess.env_boundary([binding.to_device(A)], chi, "f64", H)[0]
    g = _dev(G)
    bonds = [(r, c) for r in range(Lr) for c in range(Lc - 1)]
    got, fl = sess.bond_env([(env, r, c, g) for r, c in bonds])
    env.free()
    ref_env = api.env_boundary(A, chi, H)
    for (r, c), b in zip(bonds, got):
        check_b(b, api.bond_env(ref_env, r, c, G), TOL64)
    assert fl > 0


def test_bond_env_identity_gate_matches_site_env(sess):
    """GPU against GPU: for the identity gate b = A N with N from
    peps_site_env, at truncated chi; a Heisenberg imaginary-time gate
    against the oracle."""
    say("bond environments: identity and Heisenberg gates")
    A = make_peps(5, 5, 3, "near_product", 371)
    env = sess.env_boundary([binding.to_device(A)], 6, "f64", 4)[0]
    eye = _dev(np.eye(4).reshape(2, 2, 2, 2))
    bonds = [(0, 0), (2, 1), (4, 3)]
    got, _ = sess.bond_env([(env, r, c, eye) for r, c in bonds])
    sites, _ = sess.site_env([(env, r, c + k) for r, c in bonds for k in (0, 1)])
    for i, (r, c) in enumerate(bonds):
        for k in (0, 1):
            N = sites[2 * i + k][0].cpu().numpy()
            a = A[r][c + k].reshape(2, -1)
            assert np.abs(got[i][k].cpu().numpy() - a @ N).max() < 1e-12 * np.abs(a @ N).max()
    Gh = _heisenberg_gate(0.05)
    got, _ = sess.bond_env([(env, r, c, _dev(Gh)) for r, c in bonds])
    env.free()
    ref_env = api.env_boundary(A, 6, 4)
    for (r, c), b in zip(bonds, got):
        check_b(b, api.bond_env(ref_env, r, c, Gh), TOL64)


def test_bond_env_of_cluster_window(sess):
    """Bonds inside n = 3 windows (cut legs closed by CU_0)."""
    say("bond environments of n=3 windows")
    L, n, chi = 5, 3, 4
    A = make_peps(L, L, 2, "near_product", 381)
    sample = [(2, 2), (0, 1)]
    wins = []
    for (i, j) in sample:
        r0, r1 = cluster.window_bounds(i, n, L)
        c0, c1 = cluster.window_bounds(j, n, L)
        wins.append((0, r0, r1, c0, c1, i, j))
    envs = sess.cluster_env([binding.to_device(A)], wins, chi, "f64", 4)
    G = _gate(5)
    got, _ = sess.bond_env([(e, w[5] - w[1], w[6] - w[3], _dev(G)) for e, w in zip(envs, wins)])
    for e in envs:
        e.free()
    sep = cluster.SeparableEnv(whole_lattice(A))
    for w, b in zip(wins, got):
        _, r0, r1, c0, c1, i, j = w
        wenv = api.env_boundary(cluster.window_lattice(sep, r0, r1, c0, c1), chi, 4)
        check_b(b, api.bond_env(wenv, i - r0, j - c0, G), TOL64)


def test_bond_env_8x8_D4_chi32_sample(sess):
    """8x8, D=4, near-product, chi=32: every horizontal bond in one batched
    call, a sample against the oracle."""
    say("bond environments 8x8 D=4 chi=32")
    c = WORKLOADS["8x8_D4_chi32"]
    A = workload_peps("8x8_D4_chi32")
    env = sess.env_boundary([binding.to_device(A)], c["chi"], "f64", 4)[0]
    G = _heisenberg_gate(0.02)
    g = _dev(G)
    bonds = [(r, s) for r in range(8) for s in range(7)]
    got, _ = sess.bond_env([(env, r, s, g) for r, s in bonds])
    env.free()
    ref_env = api.env_boundary(A, c["chi"], 4)
    for k in (0, 6, 24, 55):
        r, s = bonds[k]
        check_b(got[k], api.bond_env(ref_env, r, s, G), TOL64)


def test_bond_env_fp32_form(sess):
    say("bond environments fp32")
    A = make_peps(4, 4, 3, "normal_unit", 391)
    G = _gate(7)
    env = sess.env_boundary([binding.to_device(A)], 9, "f32", 4)[0]
    got, _ = sess.bond_env([(env, 1, 1, _dev(G)), (env, 3, 2, _dev(G))])
    env.free()
    ref_env = api.env_boundary(A, 9, 4)
    check_b(got[0], api.bond_env(ref_env, 1, 1, G), 1e-4)
    check_b(got[1], api.bond_env(ref_env, 3, 2, G), 1e-4)


def test_bond_env_rejects_bad_requests(sess):
    A = make_peps(3, 3, 2, "uniform", 5)
    env = sess.env_boundary([binding.to_device(A)], 4)[0]
    g = _dev(np.eye(4))
    with pytest.raises(binding.PepsError):   # bond leaves the lattice
        sess.ctx.bond_env_raw([(env, 0, 2, g.data_ptr(), 1 << 20, 0)])
    with pytest.raises(binding.PepsError):   # no output
        sess.ctx.bond_env_raw([(env, 0, 0, g.data_ptr(), 0, 0)])
    with pytest.raises(binding.PepsError):   # no gate
        sess.ctx.bond_env_raw([(env, 0, 0, 0, 1 << 20, 0)])
    env.free()


# --- vertical bonds: the column sandwiches (environments with columns) ------

@pytest.mark.parametrize("case", [("aniso", 4, 3, 5, 3), ("normal_unit", 3, 4, 3, 4), ("normal_unit", 4, 4, 4096, 4)])
def test_vertical_site_and_bond_env_parity(sess, case):
    """dir 1: N of every site and b of both sites of every vertical bond from
    the column sandwich of the site's column, in the site's own leg order."""
    dist, Lr, Lc, chi, H = case
    say(f"vertical site/bond environments {case}")
    if dist == "aniso":
        rng = np.random.default_rng(410)
        A = [[rng.standard_normal((2, 1 if c == 0 else 2, 1 if r == 0 else 3, 1 if c == Lc - 1 else 2,
                                   1 if r == Lr - 1 else 3)) for c in range(Lc)] for r in range(Lr)]
    else:
        A = make_peps(Lr, Lc, 2, dist, 411 + Lr * Lc)
    G = _gate(Lr + Lc)
    env = sess.env_boundary([binding.to_device(A)], chi, "f64", H, columns=True)[0]
    sites = [(r, c) for r in range(Lr) for c in range(Lc)]
    Ns, _ = sess.site_env([(env, r, c, 1) for r, c in sites])
    bonds = [(r, c) for r in range(Lr - 1) for c in range(Lc)]
    bs, _ = sess.bond_env([(env, r, c, _dev(G), 1) for r, c in bonds])
    env.free()
    cols = api.env_columns(A, chi, H)
    for (r, c), g in zip(sites, Ns):
        check(g, api.site_env_columns(cols, A, r, c), TOL64)
    for (r, c), b in zip(bonds, bs):
        check_b(b, api.bond_env_vertical(cols, A, r, c, G), TOL64)


def test_vertical_needs_column_environment(sess):
    A = make_peps(3, 3, 2, "uniform", 5)
    env = sess.env_boundary([binding.to_device(A)], 4)[0]
    with pytest.raises(binding.PepsError):
        sess.ctx.site_env_raw([(env, 0, 0, 1 << 20, 1)])
    g = _dev(np.eye(4))
    with pytest.raises(binding.PepsError):
        sess.ctx.bond_env_raw([(env, 0, 0, g.data_ptr(), 1 << 20, 0, 1)])
    env.free()
    env = sess.env_boundary([binding.to_device(A)], 4, columns=True)[0]
    with pytest.raises(binding.PepsError):   # bond (2,0)-(3,0) leaves the lattice
        sess.ctx.bond_env_raw([(env, 2, 0, g.data_ptr(), 1 << 20, 0, 1)])
    env.free()


# --- the bond update's local problems with substitute tensors ----------------

@pytest.mark.parametrize("case", [("normal_unit", 3, 4, 4, 4), ("aniso", 4, 3, 5, 3)])
def test_bond_fit_parity_both_directions(sess, case):
    """N and b of both sites of every bond, with the sites replaced by
    random substitutes, from the row (dir 0) and column (dir 1) sandwiches."""
    dist, Lr, Lc, chi, H = case
    say(f"bond fit {case}")
    if dist == "aniso":
        rng = np.random.default_rng(420)
        A = [[rng.standard_normal((2, 1 if c == 0 else 2, 1 if r == 0 else 3, 1 if c == Lc - 1 else 2,
                                   1 if r == Lr - 1 else 3)) for c in range(Lc)] for r in range(Lr)]
    else:
        A = make_peps(Lr, Lc, 2, dist, 421 + Lr * Lc)
    G = _gate(11)
    env = sess.env_boundary([binding.to_device(A)], chi, "f64", H, columns=True)[0]
    ref, cols = api.env_boundary(A, chi, H), api.env_columns(A, chi, H)
    rng = np.random.default_rng(7)
    for dr in (0, 1):
        bonds = ([(r, c) for r in range(Lr) for c in range(Lc - 1)] if dr == 0
                 else [(r, c) for r in range(Lr - 1) for c in range(Lc)])
        subs = []
        for r, c in bonds:
            r2, c2 = (r, c + 1) if dr == 0 else (r + 1, c)
            subs.append((rng.standard_normal(A[r][c].shape), rng.standard_normal(A[r2][c2].shape)))
        got, _ = sess.bond_fit([(env, r, c, dr, _dev(G), _dev(s1), _dev(s2)) for (r, c), (s1, s2) in zip(bonds, subs)])
        for (r, c), (s1, s2), g in zip(bonds, subs, got):
            want = (api.bond_fit(ref, r, c, G, s1, s2) if dr == 0 else api.bond_fit_vertical(cols, r, c, G, s1, s2))
            check_b(g, want, TOL64)
    env.free()


def test_bond_fit_with_stored_tensors_equals_site_and_bond_env(sess):
    """Substitutes equal to the stored tensors: the site and bond
    environments (GPU against GPU)."""
    say("bond fit with the stored tensors")
    A = make_peps(4, 4, 2, "near_product", 431)
    env = sess.env_boundary([binding.to_device(A)], 4, "f64", 4)[0]
    G = _dev(_heisenberg_gate(0.1))
    (n1, b1, n2, b2), = sess.bond_fit([(env, 2, 1, 0, G, _dev(A[2][1]), _dev(A[2][2]))])[0]
    (bl, br), = sess.bond_env([(env, 2, 1, G)])[0]
    Ns, _ = sess.site_env([(env, 2, 1), (env, 2, 2)])
    env.free()
    for x, y in ((n1, Ns[0][0]), (n2, Ns[1][0]), (b1, bl), (b2, br)):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.abs(x - y).max() < 1e-12 * np.abs(y).max()


def test_vertical_bond_fit_with_stored_tensors_equals_site_and_bond_env(sess):
    """dir 1 (column sandwiches): substitutes equal to the stored tensors give
    the site environments and the gated-bond environments of the vertical
    bond (GPU against GPU)."""
    say("vertical bond fit with the stored tensors")
    A = make_peps(4, 4, 2, "near_product", 433)
    env = sess.env_boundary([binding.to_device(A)], 4, "f64", 4, columns=True)[0]
    G = _dev(_heisenberg_gate(0.1))
    (n1, b1, n2, b2), = sess.bond_fit([(env, 1, 2, 1, G, _dev(A[1][2]), _dev(A[2][2]))])[0]
    (bl, br), = sess.bond_env([(env, 1, 2, G, 1)])[0]
    Ns, _ = sess.site_env([(env, 1, 2, 1), (env, 2, 2, 1)])
    env.free()
    for x, y in ((n1, Ns[0][0]), (n2, Ns[1][0]), (b1, bl), (b2, br)):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.abs(x - y).max() < 1e-12 * np.abs(y).max()

"""Pins of the FP64 oracle against results fixed by the paper and by
mathematics (no GPU).  Each test names the part of the oracle it pins.
"""
import os

import numpy as np
import pytest

from oracle import api, boundary, cluster, exact, sandwich, spin, splitmix
from oracle.boundary import whole_lattice, flip_vertical, transpose_lattice
from paper_1311_6696_amd.inputs import make_peps, product_state

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _obs_close(a, b, tol):
    for k in ("sz", "bond_h", "bond_v"):
        np.testing.assert_allclose(a[k], b[k], rtol=0, atol=tol, err_msg=k)


# --- P1/P2: exact chi reproduces brute force -------------------------------

@pytest.mark.parametrize("seed", [1001, 1002, 1003])
def test_4x4_D2_matches_statevector(seed):
    """4x4, D=2, U[0,1), chi=16 (>= all caps): boundary path == 2^16 brute force."""
    A = make_peps(4, 4, 2, "uniform", seed)
    sv = exact.sv_observables(A)
    res = api.expect(api.env_boundary(A, 16))
    _obs_close(res, sv, 1e-12)
    assert abs(res["log_norm"] - np.log(sv["norm"])) < 1e-12
    assert res["sign"] == 1.0


@pytest.mark.parametrize("shape", [(3, 4, 3), (2, 5, 2), (4, 3, 2)])
def test_exact_caps_signed_states(shape):
    """Signed N(0,1) states, rectangular lattices, chi at the caps."""
    Lr, Lc, D = shape
    A = make_peps(Lr, Lc, D, "normal_unit", 17 + Lr * Lc)
    sv = exact.sv_observables(A)
    res = api.expect(api.env_boundary(A, D ** (2 * Lc)))
    _obs_close(res, sv, 1e-11)
    assert abs(res["log_norm"] - np.log(sv["norm"])) < 1e-11


def test_statevector_of_product_state():
    """The brute-force contraction itself: a D=1 PEPS is a product state."""
    A = product_state(2, 3, seed=3)
    psi = exact.statevector(A).reshape((2,) * 6)
    phi = [t.reshape(2) for row in A for t in row]
    ref = np.einsum("a,b,c,d,e,f->abcdef", *phi)
    np.testing.assert_allclose(psi, ref, atol=1e-15)


# --- P3: product states in closed form --------------------------------------

@pytest.mark.parametrize("L", [(3, 5), (4, 4), (1, 4), (5, 1)])
def test_product_state_closed_form(L):
    Lr, Lc = L
    A = product_state(Lr, Lc, seed=Lr * 10 + Lc)
    res = api.expect(api.env_boundary(A, 4))
    phi = [[t.reshape(2) for t in row] for row in A]
    n = np.array([[p @ p for p in row] for row in phi])
    sz = np.array([[(p[0] ** 2 - p[1] ** 2) / 2 / (p @ p) for p in row] for row in phi])
    sx = np.array([[p[0] * p[1] / (p @ p) for p in row] for row in phi])
    assert abs(res["log_norm"] - np.log(n).sum()) < 1e-12
    np.testing.assert_allclose(res["sz"], sz, atol=1e-14)
    np.testing.assert_allclose(res["bond_h"], sz[:, :-1] * sz[:, 1:] + sx[:, :-1] * sx[:, 1:], atol=1e-14)
    np.testing.assert_allclose(res["bond_v"], sz[:-1] * sz[1:] + sx[:-1] * sx[1:], atol=1e-14)


# --- P4: the paper's exact 4x4 energy pins operators, sign and bond list ----

def test_heisenberg_4x4_ed_value():
    ref = float(open(os.path.join(GOLDEN, "heisenberg_4x4_ed.txt")).read().split()[-1])
    e = exact.heisenberg_ground_energy(4, 4) / 16
    assert abs(e - ref) < 6e-9


def test_bond_operator_spectrum():
    """S.S on two spin-1/2: singlet -3/4, triplet +1/4 (threefold)."""
    w = np.linalg.eigvalsh(spin.bond_matrix())
    np.testing.assert_allclose(w, [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


def test_statevector_energy_matches_ed_hamiltonian():
    """Bond list and operators of the sandwich agree with the ED Hamiltonian."""
    A = make_peps(3, 3, 2, "normal_unit", 5)
    sv = exact.sv_observables(A)
    H, _ = exact.heisenberg_hamiltonian(3, 3)
    psi = exact.statevector(A)
    e_direct = psi @ (H @ psi) / (psi @ psi)
    assert abs(sv["bond_h"].sum() + sv["bond_v"].sum() - e_direct) < 1e-12


# --- P5/P6/P7: clusters ------------------------------------------------------

def test_window_equal_to_lattice_reproduces_full():
    A = make_peps(4, 4, 2, "near_product", 5)
    lat = whole_lattice(A)
    full = api.expect(api.env_boundary(lat, 8))
    out, _ = cluster.cluster_env(lat, 7, 8)
    for (i, j), (sz, right, down) in out.items():
        assert abs(sz - full["sz"][i, j]) < 1e-13
        if j < 3:
            assert abs(right - full["bond_h"][i, j]) < 1e-13
        if i < 3:
            assert abs(down - full["bond_v"][i, j]) < 1e-13


def test_n2_windows_are_exact_contractions():
    """n=2 windows at chi=D^2: no truncation, equal to one einsum of the closed window."""
    A = make_peps(4, 4, 3, "near_product", 9)
    lat = whole_lattice(A)
    out, sep = cluster.cluster_env(lat, 2, 9)
    for (i, j), (sz, right, down) in out.items():
        r0, r1 = cluster.window_bounds(i, 2, 4)
        c0, c1 = cluster.window_bounds(j, 2, 4)
        ex = exact.closed_network_observables(cluster.window_lattice(sep, r0, r1, c0, c1))
        assert abs(sz - ex["sz"][i - r0, j - c0]) < 1e-12
        if j < c1:
            assert abs(right - ex["bond_h"][i - r0, j - c0]) < 1e-12
        if i < r1:
            assert abs(down - ex["bond_v"][i - r0, j - c0]) < 1e-12


def test_cu0_positive_and_stationary():
    A = make_peps(5, 5, 3, "normal_unit", 21)
    lat = whole_lattice(A)
    sig, sweeps, delta = cluster.separable_row(lat.tau, lat.A[0], lat.lam[0], lat.rho[0])
    assert delta <= 1e-14
    assert all(np.linalg.eigvalsh(0.5 * (s + s.T)).min() > -1e-14 for s in sig)
    # stationarity: sigma_c is parallel to b_c built from the other sigmas
    P = [cluster._row_double_layer(lat.tau[c], lat.A[0][c]) for c in range(5)]
    for c in range(5):
        e = lat.lam[0]
        for k in range(c):
            e = np.einsum("lm,lmdgrs,dg->rs", e, P[k], sig[k])
        f = lat.rho[0]
        for k in range(4, c, -1):
            f = np.einsum("lmdgrs,dg,rs->lm", P[k], sig[k], f)
        b = np.einsum("lm,lmdgrs,rs->dg", e, P[c], f)
        assert np.abs(b / np.linalg.norm(b) - sig[c]).max() < 1e-12
    sep = cluster.SeparableEnv(lat)
    for grid in (sep.top, sep.bot, sep.left, sep.right):
        for row in grid:
            for s in row:
                assert np.linalg.eigvalsh(0.5 * (s + s.T)).min() > -1e-13


def test_clusters_exact_for_horizontally_decoupled_state():
    """Horizontal bonds of dimension 1: every boundary is exactly separable, so
    cluster windows of any size reproduce the brute-force values."""
    rng = np.random.default_rng(4)
    Lr, Lc, D = 4, 3, 2
    A = [[rng.random((2, 1, 1 if r == 0 else D, 1, 1 if r == Lr - 1 else D)) for c in range(Lc)]
         for r in range(Lr)]
    sv = exact.sv_observables(A)
    lat = whole_lattice(A)
    for n in (2, 3):
        out, _ = cluster.cluster_env(lat, n, 16)
        for (i, j), (sz, right, down) in out.items():
            assert abs(sz - sv["sz"][i, j]) < 1e-12
            if j < Lc - 1 and not np.isnan(right):
                assert abs(right - sv["bond_h"][i, j]) < 1e-12
            if i < Lr - 1 and not np.isnan(down):
                assert abs(down - sv["bond_v"][i, j]) < 1e-12


def test_clusters_exact_for_product_state():
    A = product_state(4, 4, seed=8)
    lat = whole_lattice(A)
    full = api.expect(api.env_boundary(lat, 1))
    out, _ = cluster.cluster_env(lat, 2, 1)
    for (i, j), (sz, right, down) in out.items():
        assert abs(sz - full["sz"][i, j]) < 1e-14


def test_window_bounds():
    assert cluster.window_bounds(0, 2, 16) == (0, 1)
    assert cluster.window_bounds(5, 4, 16) == (4, 7)
    assert cluster.window_bounds(5, 6, 16) == (3, 8)
    assert cluster.window_bounds(15, 6, 16) == (13, 15)
    assert cluster.window_bounds(1, 6, 16) == (0, 4)


# --- P8: the norm does not depend on the closing column ---------------------

def test_norm_independent_of_column():
    A = make_peps(5, 4, 2, "normal_unit", 33)
    env = api.env_boundary(A, 6, halfsweeps=3)
    T, _, _ = env.T(1)
    B, _, _ = env.B(3)
    lat = env.lat
    Lenv, Renv, sL, sR = sandwich.row_environments(T, lat.A[2], B, lat.lam[2], lat.rho[2])
    z = [np.log(abs(np.sum(Lenv[c] * Renv[c]))) + sL[c] + sR[c] for c in range(5)]
    assert np.ptp(z) < 1e-13


# --- P9: symmetries at exact chi ---------------------------------------------

def test_transpose_and_flip_symmetry():
    A = make_peps(3, 4, 2, "normal_unit", 41)
    lat = whole_lattice(A)
    ref = api.expect(api.env_boundary(lat, 64))
    tr = api.expect(api.env_boundary(transpose_lattice(lat), 64))
    np.testing.assert_allclose(tr["sz"], ref["sz"].T, atol=1e-12)
    np.testing.assert_allclose(tr["bond_h"], ref["bond_v"].T, atol=1e-12)
    np.testing.assert_allclose(tr["bond_v"], ref["bond_h"].T, atol=1e-12)
    fl = api.expect(api.env_boundary(flip_vertical(lat), 64))
    np.testing.assert_allclose(fl["sz"], ref["sz"][::-1], atol=1e-12)
    np.testing.assert_allclose(fl["bond_v"], ref["bond_v"][::-1], atol=1e-12)
    assert abs(tr["log_norm"] - ref["log_norm"]) < 1e-12


def test_gauge_invariance_truncated():
    """A bond gauge G G^-1 leaves even truncated results unchanged up to the
    ALS fixed point; at exact chi it is exact."""
    A = make_peps(3, 3, 2, "normal_unit", 43)
    rng = np.random.default_rng(0)
    G = rng.standard_normal((2, 2)) + 2 * np.eye(2)
    B = [[t.copy() for t in row] for row in A]
    B[1][1] = np.einsum("plurd,rR->pluRd", B[1][1], G)
    B[1][2] = np.einsum("Rl,plurd->pRurd", np.linalg.inv(G), B[1][2])
    a = api.expect(api.env_boundary(A, 64))
    b = api.expect(api.env_boundary(B, 64))
    _obs_close(a, b, 1e-12)


# --- P10/P11: ALS ------------------------------------------------------------

def test_als_omega_monotone_and_start_independent():
    """P10: omega never decreases over the half-sweeps, and two random starts
    reach the same fixed point: after 64 half-sweeps the observables of two
    seeds agree to 1e-11 on a strongly truncated product bond (81 -> 9) and on
    two smaller cases."""
    A = make_peps(5, 5, 3, "uniform", 7)
    lat = whole_lattice(A)
    outs = [boundary.top_boundaries(lat, 9, 16, seed) for seed in (1, 2)]
    for out in outs:
        for _, _, info in out[2:]:
            w = np.array(info.omegas)
            assert np.all(np.diff(w) >= -1e-12 * w[-1])
    for (L, D, dist, chi, s) in [(5, 3, "uniform", 9, 7), (4, 3, "near_product", 6, 8), (4, 2, "uniform", 3, 9)]:
        A = make_peps(L, L, D, dist, s)
        r = [api.expect(api.env_boundary(A, chi, 64, seed)) for seed in (1, 2)]
        _obs_close(r[0], r[1], 1e-11)


def test_als_tolerance_rule():
    """The omega stopping rule: every truncated row stops at the first
    half-sweep h >= 2 with |omega_h - omega_(h-1)| <= tol omega_h, or is
    marked not converged at the cap; with tol = 1e-15 two starts agree to
    2e-9 (omega is stationary at the fixed point, so the observables settle
    only to about sqrt(tol) times a state-dependent factor)."""
    A = make_peps(4, 4, 3, "near_product", 8)
    envs = [api.env_boundary(A, 6, 2, seed, tol=1e-15, max_halfsweeps=200) for seed in (1, 2)]
    for env in envs:
        for out in (env.top, env.bottom):
            for _, _, info in out[1:]:
                if info.exact:
                    continue
                w = info.omegas
                assert info.converged and len(w) < 200
                assert abs(w[-1] - w[-2]) <= 1e-15 * w[-1]
                assert all(abs(w[h] - w[h - 1]) > 1e-15 * w[h] for h in range(1, len(w) - 1))
    r = [api.expect(e) for e in envs]
    _obs_close(r[0], r[1], 2e-9)
    capped = api.env_boundary(A, 6, 2, 1, tol=1e-15, max_halfsweeps=5)
    infos = [x[2] for x in capped.top[1:] if not x[2].exact]
    assert infos and all(len(i.omegas) == 5 and not i.converged for i in infos)


def test_als_stationary_at_convergence():
    A = make_peps(4, 4, 3, "uniform", 8)
    lat = whole_lattice(A)
    out = boundary.top_boundaries(lat, 9, 24, 5)
    T_prev, T_new = out[1][0], out[2][0]
    # after an even number of half-sweeps the centre is site 0 and sites > 0 are right-canonical
    F = [None] * 5
    F[4] = np.ones((1, 1, 1, 1))
    for c in range(3, 0, -1):
        F[c] = boundary.env_right(F[c + 1], T_prev[c], lat.A[1][c], T_new[c])
    N0 = boundary.site_tensor(lat.lam[1].reshape(1, 1, 1, 1), T_prev[0], lat.A[1][0], F[1])
    N0 = N0 / np.linalg.norm(N0)
    assert np.abs(N0 - T_new[0]).max() < 1e-8


def test_chi_convergence_and_caps():
    A = make_peps(6, 6, 2, "normal_unit", 51)
    ref = api.expect(api.env_boundary(A, 64, halfsweeps=10))
    errs = []
    for chi in (2, 4, 8):
        r = api.expect(api.env_boundary(A, chi, halfsweeps=10))
        errs.append(np.abs(r["bond_h"] - ref["bond_h"]).max())
    assert errs[0] > errs[2]


def test_bond_caps():
    assert boundary.bond_caps(16, [16, 16, 16], [2, 2, 2, 2]) == [4, 16, 4]
    assert boundary.bond_caps(32, [256] * 7, [4] * 8) == [16, 32, 32, 32, 32, 32, 16]
    assert boundary.bond_caps(100, [16, 16], [2, 1, 2]) == [4, 4]


# --- vertical bonds from column boundaries (the sandwich along columns) -------

def _anisotropic_peps(Lr, Lc, Dh, Dv, seed):
    """Horizontal bonds of dimension Dh, vertical ones Dv (N(0,1) entries), so
    that a swapped leg pair cannot pass unnoticed."""
    rng = np.random.default_rng(seed)
    return [[rng.standard_normal((2, 1 if c == 0 else Dh, 1 if r == 0 else Dv,
                                  1 if c == Lc - 1 else Dh, 1 if r == Lr - 1 else Dv))
             for c in range(Lc)] for r in range(Lr)]


@pytest.mark.parametrize("case", [("uniform", 4, 4, 2), ("normal_unit", 3, 4, 2), ("normal_unit", 4, 3, 2),
                                  ("aniso", 3, 3, 0), ("aniso", 2, 4, 0), ("normal_unit", 1, 4, 2),
                                  ("normal_unit", 4, 1, 2)])
def test_column_vertical_bonds_match_statevector(case):
    """Exact chi: the column path's vertical bonds equal brute force, on
    rectangular, anisotropic and single-row/column lattices."""
    dist, Lr, Lc, D = case
    A = (_anisotropic_peps(Lr, Lc, 2, 3, 70 + Lr * Lc) if dist == "aniso"
         else make_peps(Lr, Lc, D, dist, 71 + Lr * Lc))
    sv = exact.sv_observables(A)
    chi = 4096
    res = api.expect(api.env_boundary(A, chi), columns=api.env_columns(A, chi))
    _obs_close(res, sv, 1e-11)
    assert abs(res["log_norm"] - np.log(sv["norm"])) < 1e-11


def test_column_boundaries_are_transposed_row_boundaries():
    """The left boundaries are the top boundaries of the transposed lattice:
    at lossless chi the ALS starts differ (other streams), so the MPS agree up
    to a gauge; their dense contractions times the log-scales agree."""
    A = make_peps(3, 4, 2, "normal_unit", 73)
    cols = api.env_columns(A, 4096)
    rows_t = api.env_boundary(transpose_lattice(whole_lattice(A)), 4096)

    def dense(T):
        x = T[0]
        for t in T[1:]:
            x = np.tensordot(x, t, axes=([-1], [0]))
        return x

    for c in range(-1, 3):
        (x, sx, _), (y, sy, _) = cols.T(c), rows_t.T(c)
        np.testing.assert_allclose(dense(x) * np.exp(sx), dense(y) * np.exp(sy), atol=1e-12)
        (x, sx, _), (y, sy, _) = cols.B(c + 2), rows_t.B(c + 2)
        np.testing.assert_allclose(dense(x) * np.exp(sx), dense(y) * np.exp(sy), atol=1e-12)


def test_column_and_two_row_paths_converge_together():
    """Truncated chi: the two routes to a vertical bond are different
    approximations; both approach the exact-chi value, and each other."""
    A = make_peps(5, 5, 2, "normal_unit", 75)
    ref = api.expect(api.env_boundary(A, 1024))["bond_v"]
    gaps, errs = [], []
    for chi in (2, 8):
        e = api.env_boundary(A, chi, halfsweeps=8)
        two = api.expect(e)["bond_v"]
        col = api.expect(e, columns=api.env_columns(A, chi, halfsweeps=8))["bond_v"]
        gaps.append(np.abs(two - col).max())
        errs.append(np.abs(col - ref).max())
    assert gaps[1] < gaps[0] and errs[1] < errs[0]
    assert errs[1] < 1e-3


# --- norm environments of single sites (the ALS update matrix N_l) ---------------

def _open_site_env(A, r0, c0):
    """Brute force N_l: site (r0, c0) replaced by the tensor that maps its
    virtual legs onto a physical index of dimension Dl Du Dr Dd; the state
    vector then holds psi_rest[sigma, k] and N = psi_rest^T psi_rest."""
    Lr, Lc = len(A), len(A[0])
    sh = A[r0][c0].shape[1:]
    K = int(np.prod(sh))
    O = np.eye(K).reshape((K,) + sh)
    B = [[O if (r, c) == (r0, c0) else A[r][c] for c in range(Lc)] for r in range(Lr)]
    i = r0 * Lc + c0
    psi = exact.statevector(B).reshape(2 ** i, K, -1)
    M = psi.transpose(0, 2, 1).reshape(-1, K)
    return M.T @ M


@pytest.mark.parametrize("case", [("normal_unit", 3, 4), ("aniso", 3, 3), ("uniform", 1, 4), ("uniform", 4, 1)])
def test_site_env_matches_brute_force(case):
    """Lossless chi: N_l / <psi|psi> and log<psi|psi> of every site equal the
    brute-force environment (corner, edge and bulk sites)."""
    dist, Lr, Lc = case
    A = (_anisotropic_peps(Lr, Lc, 2, 3, 80 + Lr * Lc) if dist == "aniso"
         else make_peps(Lr, Lc, 2, dist, 81 + Lr * Lc))
    psi = exact.statevector(A)
    Z = float(psi @ psi)
    env = api.env_boundary(A, 4096)
    for r in range(Lr):
        for c in range(Lc):
            N, lz, sgn = api.site_env(env, r, c)
            Ne = _open_site_env(A, r, c) / Z
            assert np.abs(N - Ne).max() <= 1e-12 * np.abs(Ne).max()
            assert abs(lz - np.log(Z)) < 1e-12 and sgn == 1.0


def test_site_env_symmetric_psd_and_consistent_with_sz():
    """N_l is symmetric and positive semidefinite at lossless chi; at
    truncated chi (S^z A) N A equals the row sandwich's <S^z>."""
    A = make_peps(4, 4, 2, "normal_unit", 83)
    env = api.env_boundary(A, 4096)
    N, _, _ = api.site_env(env, 1, 2)
    assert np.abs(N - N.T).max() < 1e-14 * np.abs(N).max()
    assert np.linalg.eigvalsh(N).min() > -1e-12 * np.abs(N).max()
    envt = api.env_boundary(A, 3, 4)
    res = api.expect(envt)
    for (r, c) in [(0, 0), (1, 2), (3, 3), (2, 1)]:
        N, _, sgn = api.site_env(envt, r, c)
        a = A[r][c].reshape(2, -1)
        sz_a = sandwich.apply_op(spin.SZ, A[r][c]).reshape(2, -1)
        v = np.einsum("pk,kj,pj->", sz_a, N, a) / np.einsum("pk,kj,pj->", a, N, a)
        assert abs(v - res["sz"][r, c]) < 1e-12
        assert abs(np.einsum("pk,kj,pj->", a, N, a) - sgn) < 1e-12


def _gate_applied(psi, N, i, j, G):
    """G[p, P, q, Q] on sites i < j of a 2^N state vector."""
    t = np.tensordot(G, psi.reshape((2,) * N), axes=([2, 3], [i, j]))
    return np.moveaxis(t, [0, 1], [i, j])


@pytest.mark.parametrize("case", [("normal_unit", 3, 4), ("aniso", 3, 3), ("uniform", 1, 4)])
def test_bond_env_matches_brute_force(case):
    """Lossless chi: b of both sites of every horizontal bond under a random
    two-site gate equals d<psi|G psi>/dA (brute force) over <psi|psi>."""
    dist, Lr, Lc = case
    A = (_anisotropic_peps(Lr, Lc, 2, 3, 90 + Lr * Lc) if dist == "aniso"
         else make_peps(Lr, Lc, 2, dist, 91 + Lr * Lc))
    G = np.random.default_rng(Lr * Lc).standard_normal((2, 2, 2, 2))
    psi = exact.statevector(A)
    Z = float(psi @ psi)
    N = Lr * Lc
    env = api.env_boundary(A, 4096)
    for r in range(Lr):
        for c in range(Lc - 1):
            i, j = r * Lc + c, r * Lc + c + 1
            phi = _gate_applied(psi, N, i, j, G)
            got = api.bond_env(env, r, c, G)
            for site, b in ((i, got[0]), (j, got[1])):
                rr, cc = divmod(site, Lc)
                K = int(np.prod(A[rr][cc].shape[1:]))
                O = np.eye(K).reshape((K,) + A[rr][cc].shape[1:])
                Bt = [[O if (x, y) == (rr, cc) else A[x][y] for y in range(Lc)] for x in range(Lr)]
                M = exact.statevector(Bt).reshape(2 ** site, K, -1)
                ref = np.einsum("akb,apb->pk", M, phi.reshape(2 ** site, 2, -1)) / Z
                assert np.abs(b - ref).max() <= 1e-12 * np.abs(ref).max()


def test_vertical_bond_env_and_column_site_env_match_brute_force():
    """Lossless chi: b of both sites of every vertical bond and N of every
    site, both from the column sandwiches, equal brute force (anisotropic
    bonds, so that a leg-order slip in the transposition fails)."""
    Lr, Lc = 3, 3
    A = _anisotropic_peps(Lr, Lc, 2, 3, 99)
    G = np.random.default_rng(7).standard_normal((2, 2, 2, 2))
    psi = exact.statevector(A)
    Z = float(psi @ psi)
    N = Lr * Lc
    cols = api.env_columns(A, 4096)

    def open_M(rr, cc):
        K = int(np.prod(A[rr][cc].shape[1:]))
        O = np.eye(K).reshape((K,) + A[rr][cc].shape[1:])
        Bt = [[O if (x, y) == (rr, cc) else A[x][y] for y in range(Lc)] for x in range(Lr)]
        return exact.statevector(Bt).reshape(2 ** (rr * Lc + cc), K, -1)

    for r in range(Lr):
        for c in range(Lc):
            M = open_M(r, c)
            Mm = M.transpose(0, 2, 1).reshape(-1, M.shape[1])
            Nc, _, _ = api.site_env_columns(cols, A, r, c)
            assert np.abs(Nc - Mm.T @ Mm / Z).max() <= 1e-12 * np.abs(Nc).max()
    for r in range(Lr - 1):
        for c in range(Lc):
            i, j = r * Lc + c, (r + 1) * Lc + c
            phi = _gate_applied(psi, N, i, j, G)
            bl, br = api.bond_env_vertical(cols, A, r, c, G)
            for site, b in ((i, bl), (j, br)):
                M = open_M(*divmod(site, Lc))
                ref = np.einsum("akb,apb->pk", M, phi.reshape(2 ** site, 2, -1)) / Z
                assert np.abs(b - ref).max() <= 1e-12 * np.abs(ref).max()


def test_bond_env_identity_gate_is_N_times_A():
    """Truncated chi: for the identity gate b[p, k'] = sum_k A[p, k] N[k, k']
    for both sites (the scalings of the bond and site environments agree;
    truncated boundaries need not be symmetric under ket <-> bra, so the
    contraction runs over N's ket index)."""
    A = make_peps(4, 4, 2, "normal_unit", 93)
    env = api.env_boundary(A, 3, 4)
    eye = np.eye(4).reshape(2, 2, 2, 2)
    for (r, c) in [(0, 0), (1, 2), (3, 1)]:
        bl, br = api.bond_env(env, r, c, eye)
        for b, cc in ((bl, c), (br, c + 1)):
            Nm, _, sgn = api.site_env(env, r, cc)
            a = A[r][cc].reshape(2, -1)
            assert np.abs(b - a @ Nm).max() < 1e-12 * np.abs(b).max()


def test_bond_fit_with_substitutes_matches_brute_force():
    """The bond update's two local problems with the sites replaced by
    random S1, S2: N and b of each site equal the brute-force norm
    environment of psi' and d<psi'|G psi>/dS up to one common factor per
    site (the factor the solve S = b N^-1 does not see); with S = A they
    equal the site and bond environments."""
    Lr, Lc = 3, 4
    A = make_peps(Lr, Lc, 2, "normal_unit", 101)
    G = np.random.default_rng(3).standard_normal((2, 2, 2, 2))
    env = api.env_boundary(A, 4096)
    r, c = 1, 1
    N1, b1, N2, b2 = api.bond_fit(env, r, c, G, A[r][c], A[r][c + 1])
    bl, br = api.bond_env(env, r, c, G)
    assert np.abs(N1 - api.site_env(env, r, c)[0]).max() < 1e-13
    assert np.abs(N2 - api.site_env(env, r, c + 1)[0]).max() < 1e-13
    assert np.abs(b1 - bl).max() < 1e-13 and np.abs(b2 - br).max() < 1e-13
    rng = np.random.default_rng(4)
    S1, S2 = rng.standard_normal(A[r][c].shape), rng.standard_normal(A[r][c + 1].shape)
    N1, b1, N2, b2 = api.bond_fit(env, r, c, G, S1, S2)
    psi = exact.statevector(A)
    i, j = r * Lc + c, r * Lc + c + 1
    phi = _gate_applied(psi, Lr * Lc, i, j, G)
    for site, other, Sother, N, b in ((i, (r, c + 1), S2, N1, b1), (j, (r, c), S1, N2, b2)):
        Ap = [list(row) for row in A]
        Ap[other[0]][other[1]] = Sother
        rr, cc = divmod(site, Lc)
        K = int(np.prod(A[rr][cc].shape[1:]))
        O = np.eye(K).reshape((K,) + A[rr][cc].shape[1:])
        Bt = [[O if (x, y) == (rr, cc) else Ap[x][y] for y in range(Lc)] for x in range(Lr)]
        M = exact.statevector(Bt).reshape(2 ** site, K, -1)
        Mm = M.transpose(0, 2, 1).reshape(-1, K)
        Nex = Mm.T @ Mm
        bex = np.einsum("akb,apb->pk", M, phi.reshape(2 ** site, 2, -1))
        f = np.sum(Nex * N) / np.sum(N * N)
        assert np.abs(N * f - Nex).max() <= 1e-12 * np.abs(Nex).max()
        assert np.abs(b * f - bex).max() <= 1e-12 * np.abs(bex).max()


def test_bond_fit_vertical_with_substitutes_matches_brute_force():
    """The vertical bond's two local problems from the column sandwiches
    (anisotropic bonds, so a swapped leg pair in the transposition fails):
    with S = A they equal the column site and bond environments; with random
    S1 on (r, c) and S2 on (r+1, c) N and b of each site equal the brute-force
    norm environment of psi' and d<psi'|G psi>/dS up to one common factor per
    site."""
    Lr, Lc = 3, 3
    A = _anisotropic_peps(Lr, Lc, 2, 3, 103)
    G = np.random.default_rng(5).standard_normal((2, 2, 2, 2))
    cols = api.env_columns(A, 4096)
    psi = exact.statevector(A)
    for (r, c) in [(0, 1), (1, 0), (1, 2)]:
        N1, b1, N2, b2 = api.bond_fit_vertical(cols, r, c, G, A[r][c], A[r + 1][c])
        bl, br = api.bond_env_vertical(cols, A, r, c, G)
        assert np.abs(N1 - api.site_env_columns(cols, A, r, c)[0]).max() < 1e-13
        assert np.abs(N2 - api.site_env_columns(cols, A, r + 1, c)[0]).max() < 1e-13
        assert np.abs(b1 - bl).max() < 1e-13 and np.abs(b2 - br).max() < 1e-13
        rng = np.random.default_rng(10 + r * Lc + c)
        S1, S2 = rng.standard_normal(A[r][c].shape), rng.standard_normal(A[r + 1][c].shape)
        N1, b1, N2, b2 = api.bond_fit_vertical(cols, r, c, G, S1, S2)
        i, j = r * Lc + c, (r + 1) * Lc + c
        phi = _gate_applied(psi, Lr * Lc, i, j, G)
        for site, other, Sother, N, b in ((i, (r + 1, c), S2, N1, b1), (j, (r, c), S1, N2, b2)):
            Ap = [list(row) for row in A]
            Ap[other[0]][other[1]] = Sother
            rr, cc = divmod(site, Lc)
            K = int(np.prod(A[rr][cc].shape[1:]))
            O = np.eye(K).reshape((K,) + A[rr][cc].shape[1:])
            Bt = [[O if (x, y) == (rr, cc) else Ap[x][y] for y in range(Lc)] for x in range(Lr)]
            M = exact.statevector(Bt).reshape(2 ** site, K, -1)
            Mm = M.transpose(0, 2, 1).reshape(-1, K)
            Nex = Mm.T @ Mm
            bex = np.einsum("akb,apb->pk", M, phi.reshape(2 ** site, 2, -1))
            f = np.sum(Nex * N) / np.sum(N * N)
            assert f > 0
            assert np.abs(N * f - Nex).max() <= 1e-12 * np.abs(Nex).max()
            assert np.abs(b * f - bex).max() <= 1e-12 * np.abs(bex).max()


# --- boundary fidelity ---------------------------------------------------------

def _dense_mps(T):
    x = T[0]
    for t in T[1:]:
        x = np.tensordot(x, t, axes=([-1], [0]))
    return x.reshape(-1)


def test_boundary_overlap_is_dense_inner_product_and_unit_norm():
    """The overlap chain equals the inner product of the fully contracted
    boundaries, and every stored boundary has unit norm."""
    A = make_peps(4, 4, 2, "normal_unit", 95)
    e1, e2 = api.env_boundary(A, 6, seed=5), api.env_boundary(A, 3, seed=6)
    for k in range(1, 4):
        X, Y = e1.T(k - 1)[0], e2.T(k - 1)[0]
        assert abs(boundary.mps_overlap(X, Y) - _dense_mps(X) @ _dense_mps(Y)) < 1e-13
        assert abs(boundary.mps_overlap(X, X) - 1.0) < 1e-13
        X, Y = e1.B(4 - k)[0], e2.B(4 - k)[0]
        assert abs(boundary.mps_overlap(X, Y) - _dense_mps(X) @ _dense_mps(Y)) < 1e-13


def test_boundary_fidelity_one_at_lossless_chi_below_one_truncated():
    """Lossless chi from two different ALS starts: the same boundary in
    another gauge, f = 1; truncated boundaries have f < 1, closer to 1 at
    larger chi."""
    A = make_peps(5, 5, 2, "normal_unit", 97)
    e1, e2 = api.env_boundary(A, 1024, seed=1), api.env_boundary(A, 1024, seed=2)
    for side in (0, 1):
        for k in range(1, 5):
            assert abs(1.0 - api.boundary_fidelity(e1, e2, side, k)) < 1e-12
    worst = [max(1.0 - api.boundary_fidelity(e1, api.env_boundary(A, chi), 0, k) for k in range(1, 5))
             for chi in (2, 4, 8)]
    assert worst[0] > worst[1] > worst[2] > 0.0


# --- P12/P13 ------------------------------------------------------------------

def test_bounds_at_exact_chi():
    A = make_peps(3, 4, 2, "normal_unit", 61)
    res = api.expect(api.env_boundary(A, 64))
    assert np.all(np.abs(res["sz"]) <= 0.5 + 1e-12)
    for k in ("bond_h", "bond_v"):
        assert np.all(res[k] >= -0.75 - 1e-12) and np.all(res[k] <= 0.25 + 1e-12)


def test_near_product_is_ferromagnetic():
    A = make_peps(4, 4, 4, "near_product", 1002)
    res = api.expect(api.env_boundary(A, 16))
    for k in ("bond_h", "bond_v"):
        assert np.all(np.abs(res[k] - 0.25) < 0.08)


# --- SplitMix64 -----------------------------------------------------------------

def test_splitmix64_reference_sequence():
    """First outputs of SplitMix64 seeded with 1234567 (widely reproduced
    reference values of the published generator)."""
    s = 1234567
    got = []
    for _ in range(3):
        s = (s + splitmix.GAMMA) & splitmix.MASK
        got.append(splitmix.mix(s))
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_splitmix_uniform_vectorised_matches_scalar():
    q = splitmix.als_stream(1, 3, 2)
    s = splitmix.stream_state(7, q)
    ref = [((splitmix.mix(s + (n + 1) * splitmix.GAMMA) >> 11) * 2.0 ** -53) * 2 - 1 for n in range(50)]
    np.testing.assert_array_equal(splitmix.uniform(7, q, 50), np.array(ref))

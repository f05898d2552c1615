"""Top-level oracle calls mirroring the C ABI: environment, expectation values
and cluster windows.  Test infrastructure only (see the package docstring).

* ``env_boundary`` - boundaries from the top and from the bottom with bond chi
  (Sec. 2, the sandwich contraction from both sides).
* ``expect`` - log <psi|psi> and its sign from the row in the centre, <S^z>
  on every site from its row sandwich, horizontal bond energies from the row
  sandwich and vertical ones from the two-row sandwich (readings, see
  ``sandwich``).
* ``env_columns`` - boundaries from the left and from the right: the top and
  bottom boundaries of the transposed lattice (the same sandwich contraction
  run along the other lattice direction, Sec. 2).  Passed to ``expect``, they
  give the vertical bond energies from single-column sandwiches instead of
  two-row sandwiches.
* ``site_env`` - norm environment N_l of one site (Sec. 2, the matrix of
  the ALS tensor update) from its row sandwich, scaled to A N A = +-1, with
  the log of the scale.
* ``bond_env`` - right-hand sides b_l of the ALS update of a horizontal
  bond under a two-site gate (Sec. 2), in the scaling of ``site_env``.
* ``cluster_env`` - per-site n x n windows closed by CU_0 separable
  boundaries (``cluster``), Sec. 5.3.
"""
from dataclasses import dataclass

import numpy as np

from .boundary import flip_vertical, top_boundaries, transpose_lattice, whole_lattice, Lattice
from .sandwich import bond_gate_environment, row_observables, site_environment, two_row_observables

DEFAULT_SEED = 0x13116696
DEFAULT_HALFSWEEPS = 4


@dataclass
class Env:
    lat: Lattice
    top: list      # top[r+1] = (tensors, log_scale, info) of T_r, r = -1..Lr-2
    bottom: list   # bottom[k] = boundary of the flipped lattice, k-1 rows absorbed
    chi: int

    def T(self, r):
        """Top boundary with rows 0..r absorbed (r = -1 is the top closing)."""
        return self.top[r + 1]

    def B(self, r):
        """Bottom boundary with rows r..Lr-1 absorbed (r = Lr is the closing),
        tensors [o, d, g, o'] with d,g the down legs of row r-1."""
        return self.bottom[self.lat.rows - r]


def env_boundary(lat_or_A, chi, halfsweeps=DEFAULT_HALFSWEEPS, seed=DEFAULT_SEED, tol=0.0, max_halfsweeps=None):
    """Top and bottom boundaries.  ``halfsweeps`` ALS half-sweeps per
    truncated row; with ``tol`` > 0 the sweeps go on until the squared centre
    norm settles to ``tol`` (relative) or ``max_halfsweeps`` have run."""
    lat = lat_or_A if isinstance(lat_or_A, Lattice) else whole_lattice(lat_or_A)
    top = top_boundaries(lat, chi, halfsweeps, seed, 0, tol, max_halfsweeps)
    bottom = top_boundaries(flip_vertical(lat), chi, halfsweeps, seed, 1, tol, max_halfsweeps)
    return Env(lat, top, bottom, chi)


def env_columns(lat_or_A, chi, halfsweeps=DEFAULT_HALFSWEEPS, seed=DEFAULT_SEED, tol=0.0, max_halfsweeps=None):
    """Left and right boundaries of a lattice, as an ``Env`` of its transpose:
    its T(c) holds columns 0..c absorbed from the left, its B(c) columns
    c..Lc-1 absorbed from the right.  ALS start streams use side 2 (from the
    left) and side 3 (from the right), so that they differ from the streams
    of the row boundaries."""
    lat = lat_or_A if isinstance(lat_or_A, Lattice) else whole_lattice(lat_or_A)
    tl = transpose_lattice(lat)
    top = top_boundaries(tl, chi, halfsweeps, seed, 2, tol, max_halfsweeps)
    bottom = top_boundaries(flip_vertical(tl), chi, halfsweeps, seed, 3, tol, max_halfsweeps)
    return Env(tl, top, bottom, chi)


def expect(env, rows=None, columns=None):
    """Observables of an environment; ``rows`` limits the single-row sandwiches.

    With ``columns`` (from ``env_columns`` of the same lattice), the vertical
    bond (r, c)-(r+1, c) is the horizontal bond (c, r)-(c, r+1) of the
    transposed lattice, taken from its single-row sandwich of row c; the
    two-row sandwiches are then not formed."""
    lat = env.lat
    Lr, Lc = lat.rows, lat.cols
    sz = np.full((Lr, Lc), np.nan)
    bh = np.full((Lr, max(Lc - 1, 0)), np.nan)
    bv = np.full((max(Lr - 1, 0), Lc), np.nan)
    log_norm, sign = None, None
    rc = Lr // 2
    for r in (range(Lr) if rows is None else rows):
        T, sT, _ = env.T(r - 1)
        B, sB, _ = env.B(r + 1)
        s, h, Z, sLR, _ = row_observables(T, lat.A[r], B, lat.lam[r], lat.rho[r])
        sz[r], bh[r] = s, h
        if r == rc:
            log_norm = sT + sB + sLR + np.log(abs(Z))
            sign = 1.0 if Z >= 0 else -1.0
    if columns is not None:
        tl = columns.lat
        assert tl.rows == Lc and tl.cols == Lr, "column environment of another lattice"
        for c in range(Lc):
            T, _, _ = columns.T(c - 1)
            B, _, _ = columns.B(c + 1)
            _, h, _, _, _ = row_observables(T, tl.A[c], B, tl.lam[c], tl.rho[c])
            bv[:, c] = h
        return dict(log_norm=log_norm, sign=sign, sz=sz, bond_h=bh, bond_v=bv)
    for r in (range(Lr - 1) if rows is None else [x for x in rows if x < Lr - 1]):
        T, _, _ = env.T(r - 1)
        B, _, _ = env.B(r + 2)
        bv[r] = two_row_observables(T, lat.A[r], lat.A[r + 1], B, lat.lam[r], lat.rho[r],
                                    lat.lam[r + 1], lat.rho[r + 1])
    return dict(log_norm=log_norm, sign=sign, sz=sz, bond_h=bh, bond_v=bv)


def site_env(env, r, c):
    """(N, log_z, sign) of site (r, c): N scaled so that sum_p A N A = sign,
    log_z the log of |<psi|psi>| as this row's sandwich estimates it (so the
    unscaled environment is sign * exp(log_z) * N)."""
    lat = env.lat
    T, sT, _ = env.T(r - 1)
    B, sB, _ = env.B(r + 1)
    N, lz, sgn = site_environment(T, lat.A[r], B, lat.lam[r], lat.rho[r], c)
    return N, lz + sT + sB, sgn


def bond_env(env, r, c, G):
    """(b_left, b_right) of the horizontal bond (r, c)-(r, c+1) under the
    two-site gate G[p, P, q, Q], each (d, Dl Du Dr Dd), in the scaling of
    ``site_env`` of the same site (G = 1 gives b = N A)."""
    lat = env.lat
    T, _, _ = env.T(r - 1)
    B, _, _ = env.B(r + 1)
    return bond_gate_environment(T, lat.A[r], B, lat.lam[r], lat.rho[r], c, G)


def boundary_fidelity(env_a, env_b, side, k):
    """Fidelity of two environments' boundaries of one lattice after k
    absorbed rows: side 0 from the top (T(k-1)), side 1 from the bottom
    (B(Lr-k))."""
    from .boundary import boundary_fidelity as fid
    Lr = env_a.lat.rows
    X = env_a.T(k - 1)[0] if side == 0 else env_a.B(Lr - k)[0]
    Y = env_b.T(k - 1)[0] if side == 0 else env_b.B(Lr - k)[0]
    return fid(X, Y)


def _from_transposed(x, shape, matrix):
    """A site quantity computed on the transposed lattice (legs l, u, r, d of
    the transpose = u, l, d, r of the site) back in the site's own order."""
    d, Dl, Du, Dr, Dd = shape
    if matrix:
        return x.reshape(Du, Dl, Dd, Dr, Du, Dl, Dd, Dr).transpose(1, 0, 3, 2, 5, 4, 7, 6).reshape(x.shape)
    return x.reshape(d, Du, Dl, Dd, Dr).transpose(0, 2, 1, 4, 3).reshape(x.shape)


def site_env_columns(columns, A, r, c):
    """``site_env`` of site (r, c) from the column sandwich of column c
    (``columns`` from ``env_columns``), in the site's own leg order."""
    N, lz, sgn = site_env(columns, c, r)
    return _from_transposed(N, A[r][c].shape, True), lz, sgn


def bond_env_vertical(columns, A, r, c, G):
    """``bond_env`` of the vertical bond (r, c)-(r+1, c) from the column
    sandwich of column c: (b of (r, c), b of (r+1, c)), G's first index pair
    on (r, c), each in the site's own leg order."""
    bl, br = bond_env(columns, c, r, G)
    return _from_transposed(bl, A[r][c].shape, False), _from_transposed(br, A[r + 1][c].shape, False)


def bond_fit(env, r, c, G, S1, S2):
    """(N1, b1, N2, b2) of fitting G psi on the horizontal bond (r, c)-(r, c+1)
    with the sites replaced by S1, S2 (``bond_fit_environments``)."""
    lat = env.lat
    T, _, _ = env.T(r - 1)
    B, _, _ = env.B(r + 1)
    from .sandwich import bond_fit_environments
    return bond_fit_environments(T, lat.A[r], B, lat.lam[r], lat.rho[r], c, G, S1, S2)


def bond_fit_vertical(columns, r, c, G, S1, S2):
    """``bond_fit`` of the vertical bond (r, c)-(r+1, c) from the column
    sandwich of column c; S1, S2 and the results in the sites' own order."""
    N1, b1, N2, b2 = bond_fit(columns, c, r, G, S1.transpose(0, 2, 1, 4, 3), S2.transpose(0, 2, 1, 4, 3))
    return (_from_transposed(N1, S1.shape, True), _from_transposed(b1, S1.shape, False),
            _from_transposed(N2, S2.shape, True), _from_transposed(b2, S2.shape, False))


def energy(res):
    """Total Heisenberg energy sum of bond terms (eq. HeisenbergH)."""
    return float(np.nansum(res["bond_h"]) + np.nansum(res["bond_v"]))

"""Seeded synthetic PEPS inputs (shared by tests, bench and smoke).

Holds no step of the contraction method: it only draws site tensors.  The
paper's benchmark states (optimised Heisenberg/Ising PEPS) are not available,
so these stand in for them with the same shapes: square open-boundary
lattices, physical dimension 2, bulk bond D, edge legs of dimension 1.

Site tensors are float64 arrays A[p, l, u, r, d] in C order; sites are drawn
row-major from one ``numpy.random.Generator(PCG64(seed))``.

Distributions
-------------
uniform       i.i.d. U[0, 1)                       (all-positive states)
near_product  A[0,0,0,0,0] = 1, every other entry 0.1 * N(0, 1)
normal_unit   i.i.d. N(0, 1), then each tensor scaled to unit Frobenius norm
"""
import numpy as np


def site_shape(r, c, Lr, Lc, d, D):
    return (d, 1 if c == 0 else D, 1 if r == 0 else D,
            1 if c == Lc - 1 else D, 1 if r == Lr - 1 else D)


def draw_site(rng, shape, dist):
    if dist == "uniform":
        return rng.random(shape)
    if dist == "near_product":
        t = 0.1 * rng.standard_normal(shape)
        t[(0,) * len(shape)] = 1.0
        return t
    if dist == "normal_unit":
        t = rng.standard_normal(shape)
        return t / np.sqrt(np.sum(t * t))
    raise ValueError(f"unknown distribution {dist!r}")


def make_peps(Lr, Lc, D, dist="uniform", seed=0, d=2, rng=None):
    """List of Lr rows of Lc site tensors."""
    rng = rng if rng is not None else np.random.Generator(np.random.PCG64(seed))
    return [[draw_site(rng, site_shape(r, c, Lr, Lc, d, D), dist) for c in range(Lc)]
            for r in range(Lr)]


def product_state(Lr, Lc, seed=0):
    """D = 1 PEPS: one random 2-vector per site (for closed-form checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [[rng.standard_normal((2, 1, 1, 1, 1)) for _ in range(Lc)] for _ in range(Lr)]


# Seeded workloads with the shapes of the paper's benchmark states, named by
# lattice, bond dimension and chi: (lattice side, D, distribution, chi, seed).
WORKLOADS = {
    "4x4_D2_exact": dict(L=4, D=2, dist="uniform", chi=16, seed=1001,
                         note="4x4, D=2, U[0,1), chi=16 (exact); checked against the 2^16 state vector"),
    "8x8_D4_chi32": dict(L=8, D=4, dist="near_product", chi=32, seed=1002,
                         note="8x8, D=4, near-product signed, chi=32, plain FP64"),
    "10x10_D6_chi72": dict(L=10, D=6, dist="normal_unit", chi=72, seed=1003,
                           note="10x10, D=6, N(0,1) unit-norm tensors, chi=72, precision form"),
    "16x16_D6_clusters": dict(L=16, D=6, dist="near_product", chi=36, seed=1004, ns=(2, 4, 6),
                              note="16x16, D=6, near-product, chi=36, n x n clusters n in {2,4,6}"),
}


def workload_peps(name, seed=None):
    c = WORKLOADS[name]
    return make_peps(c["L"], c["L"], c["D"], c["dist"], c["seed"] if seed is None else seed)


def batched_instances(count=32, seed=1005, Ls=range(6, 13), Ds=(3, 4, 5, 8)):
    """``count`` independent PEPS of seeded sizes (L in 6..12, D in {3,4,5,8}).

    One generator draws all (L, D) pairs first, then the tensors instance by
    instance (sites row-major), entries U[0, 1); chi = D^2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls, Ds = list(Ls), list(Ds)
    pairs = [(int(Ls[rng.integers(len(Ls))]), int(Ds[rng.integers(len(Ds))])) for _ in range(count)]
    insts = [make_peps(L, L, D, "uniform", rng=rng) for (L, D) in pairs]
    return pairs, insts

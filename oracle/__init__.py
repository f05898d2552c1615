"""Plain FP64 CPU oracle for the boundary-MPS environment of a finite PEPS.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: it is written from the paper (Lubasch, Cirac, Banuls, "Unifying
Projected Entangled Pair States contractions", arXiv:1311.6696) with NumPy
``einsum``/``tensordot`` and LAPACK QR as its only library primitives.

Modules
-------
spin       spin-1/2 operators and the Heisenberg bond term (eq. HeisenbergH)
splitmix   SplitMix64 counter generator used for the ALS start tensors
exact      state-vector / direct-einsum references and Lanczos ED (pins only)
boundary   boundary-MPS row absorption with ALS truncation (Sec. 2, fig. Sandwich)
sandwich   one-row and two-row sandwiches -> norm, <Sz>, bond energies
cluster    CU_0 separable boundaries and n x n cluster windows (Sec. 5.1-5.3)
api        the three top-level calls mirrored by the C ABI

Parity status: every function is pinned by a ``-m "not gpu"`` test against
an independent result (brute force, closed form, ED value printed in the
paper, limiting case or invariant) except the truncated-chi values, which are
pinned only through invariants (ALS monotonicity, start independence at
convergence, chi-convergence); see the test files for the pin of each
function.
"""

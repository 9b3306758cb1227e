"""Oracle: a plain, slow, FP64 CPU reference of the Lindblad MPO-TEBD step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP library
(different language, different basis: this package works in the computational
basis |ket><bra| per site, the library in the normalised Pauli basis).

Sources (Landa & Misguich, arXiv:2203.05871):
  model.py         Lindbladian of Eqs. (dtrho), (H0), (K_def), (D0)-(D2),
                   split into per-bond generators and exponentiated
  tebd.py          vectorised density matrix as an MPS (Eq. mpo_def, App. A),
                   two-site gates, truncation by the more severe of the
                   discarded-weight cutoff and the maximal bond dimension
                   (App. B), trace forcing (App. B, Sec. 6 parameters),
                   1Q/2Q observables (Eqs. mu, 2Qdef), trace (Sec. 2.4)
  dense.py         brute-force 4^N references: the same Trotter product
                   without truncation, and exact exponentiation of the full
                   Liouvillian (the paper's brute-force comparison, Sec. 3.2)
  adjoint.py       parameter gradients of a final-time expectation value by
                   the adjoint (co-state) method on the MPS: transposed gates
                   carry the co-state back, every gate contributes the trace
                   of its Frechet-derivative factor with the two-site
                   transition density of state and co-state
  closed_forms.py  textbook closed forms used as pins: single-qubit Bloch
                   equations and their steady state, the one-excitation
                   sector of the XY chain (Sec. 3.2, free-fermion picture)

Parity status: every function is pinned by tests/test_oracle_*.py against the
closed forms, the dense references, or brute force.  The truncated regime
(chi below 4^floor(N/2)) has no closed form; it is pinned by convergence to
the dense result as chi grows, by the exact Delta=0 symmetry, and by the
truncation rule checked on hand-made spectra.
"""

"""CPU oracle for exact effective resistances -- TEST INFRASTRUCTURE ONLY.

Only the test suite (``tests/``), the package smoke check
(``__graft_entry__.smoke``) and the benchmark's ``cpu_baseline`` leg may import
anything from here. The product path (the HIP library and its Python binding)
never imports, links or calls it, and the two share no code: the only common
dependency is the seeded input generator module ``synth``, which holds no
arithmetic of the method.

What it computes is the plain definition, not the paper's algorithm. The paper
proves (Section IV-A, Theorem 3) that the implicit sweep equals the exact
effective resistance up to rounding, so the oracle evaluates

    R_uv = (e_u - e_v)^T  L_r^{-1}  (e_u - e_v)          (Section II-A, eq 2 / eq 15)

on the grounded Laplacian ``L_r`` of ``L_G = sum_e w_e e_e e_e^T`` (eq 1), with
``e_g := 0`` for the ground node (eq 4). Modules:

  laplacian  eq 1 and grounding
  dense      eq 2 by dense Cholesky (n up to a few thousand), pseudo-inverse cross-check
  sparse     eq 2 per pair by a sparse LU with the oracle's own nested dissection
             and extended-precision iterative refinement (any n, sampled pairs)
  exact      exact rational R by Cramer's rule on the grounded Laplacian, and by
             spanning-tree enumeration (Kirchhoff), for tiny graphs
  symbolic   elimination tree, factor pattern, supernodes and reach sets from their
             definitions (Lemma 1, Definition 2, Algorithm 3)
  factor     oracles that take a factor L D L^T as data: per-pair LSolve (the
             paper's accuracy protocol, Section V-A) and the dense columns of
             Z = D^{-1/2} L^{-1} that the sweep produces implicitly (Lemma 3)
  sparsify   Algorithm 1 (sampling edges by w_e R_e) with a counter-based
             generator, for the device sparsifier
"""
from . import laplacian, dense, sparse, exact, symbolic, factor, sparsify  # noqa: F401

__all__ = ["laplacian", "dense", "sparse", "exact", "symbolic", "factor", "sparsify"]

"""FP64 CPU oracle for preconditioned data sparsification (arXiv 1511.00152).

TEST INFRASTRUCTURE ONLY.  The product path (the HIP library and its Python
binding) never imports, links or runs anything in this package; only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` do.

Two tiers, both written from the paper:

* ``oracle_def`` -- literal matrices for tiny sizes: an explicit normalized
  Hadamard matrix, explicit p x m sampling matrices R_i, and the estimators
  typed in as the paper displays them.
* ``ref`` -- a plain C implementation (``ref.c``, FP64, OpenMP over samples)
  of the same steps at useful sizes, pinned against ``oracle_def`` and
  against invariants the paper fixes.

Parity status per function is listed in ``ref.py``'s module docstring.
"""

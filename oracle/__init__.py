"""CPU FP64 oracle for the PIE / MLFMA matrix-vector product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
shares no code with the HIP path: the two meet only through the seeded inputs
of the top-level ``synth`` module.

Contents, each written from the paper (arXiv:1806.04164) and plain mathematics:

* ``mesh``     RWG (edge) and pulse (triangle) discretisation of Section 2.
* ``quad``     the 7-point degree-5 triangle rule used for every integral.
* ``potint``   closed-form integrals of 1/R and (r'-rho)/R over a triangle
               (singularity extraction for touching triangle pairs).
* ``mom``      the dense Galerkin method-of-moments matrix of Eqs. (1)-(2)
               (the plain definition the MLFMA approximates), right-hand
               sides and far fields.
* ``octree``   cubic-box clustering, near lists, interaction lists (Sec. 3).
* ``mlfma``    the MLFMA steps of Section 3 in FP64: radiation patterns,
               aggregation, translation with Eqs. (4)-(5), disaggregation.
* ``gmres``    plain restarted GMRES (Section 4).
* ``schwarz``  restricted additive Schwarz preconditioner over finest-box
               near neighbourhoods (a reading: the paper names no
               preconditioner).
* ``mie``      Mie series for a PEC sphere (Section 4's analytic reference).

Parity status of each function is stated in its docstring; anything without
an independent pin says "parity unpinned".
"""

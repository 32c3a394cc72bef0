"""FP64 CPU oracle for the nodal DG velocity-stress elastic-wave right-hand
side and its low-storage Runge-Kutta update.

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product path: only
the test-suite, the package smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the HIP library (no common
kernels, headers, helpers or tables); the only common inputs come from the
``synth`` module of seeded generators, which holds none of the method's
arithmetic.

The mounted paper (sparse-grid noise reduction for particle-in-cell) states
no discontinuous-Galerkin method, so every function here follows a standard
published formulation, cited by name:

* [HW08]  Hesthaven & Warburton, *Nodal Discontinuous Galerkin Methods*,
  Springer 2008 -- orthonormal simplex basis (Ch. 6 and 10), strong-form
  DG with LIFT (Ch. 2-3 and 10).
* [CHW17] Chan, Hewett & Warburton, "Weight-adjusted discontinuous Galerkin
  methods: curvilinear meshes", SISC 2017; [C18] Chan, "Weight-adjusted DG
  methods: matrix-valued weights and elastic wave propagation in
  heterogeneous media", IJNME 2018 -- the weight-adjusted mass inverse.
* [WSG10] Wilcox, Stadler, Burstedde & Ghattas, "A high-order DG method
  for wave propagation through coupled elastic-acoustic media", JCP 2010
  -- the exact-Riemann (upwind) elastic flux.
* [CK94]  Carpenter & Kennedy, "Fourth-order 2N-storage Runge-Kutta
  schemes", NASA TM-109112, 1994 -- LSRK(5,4).

Parity status per function is listed in the header of each module.
"""

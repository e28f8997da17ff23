"""FP64 CPU oracle for the EMU deformation-space quasi-static solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or executes anything in this package; only the
tests, the smoke check and the benchmark's CPU-baseline leg use it.

Everything here is plain NumPy/SciPy in float64, written from the paper's
method section (Sec. 3, 3.1, 3.2, 3.2.1, 3.4) with the readings that the design
notes list.  Modules:

* ``material``  -- stable Neo-Hookean + linear fiber energy, stress and Hessian
  (F form), and the symmetric 6-vector basis used by the S form.
* ``mesh``      -- orientation, hat gradients, volumes, ACAP weights, the
  weighted Laplacian, its factorization and eigenmodes (eq. defograd,
  eq. ACAPEnergy, eq. acap, eq. low-rank).
* ``emu``       -- the S-form EMU quasi-Newton solver (Sec. 3.2.1, Algorithm 1).
* ``fem``       -- two independent q-space Newton solvers: the Moreau-envelope
  FEM whose minimizer equals EMU's, and plain FEM (the alpha -> infinity limit).
* ``dense``     -- brute-force dense F-form Newton for meshes of a few tets
  (eq. full-Hessian).
* ``closed``    -- closed-form special cases.
* ``adjoint``   -- q-space adjoint of the equilibrium w.r.t. muscle activations.
"""

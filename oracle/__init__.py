"""FP64 CPU oracle of the generalized-polynomial lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
in this package.  The product (``paper_1510_07328_amd``) never imports it, and it
never imports the product: the two share no code, tables or constants.

Modules:
    theory   -- weight moments, polynomial coefficients, P and A tensors, velocity
                sets and their quadrature weights (numpy, float64)
    lbm      -- ctypes front end of lbm_oracle.c, the plain C FP64 lattice BGK run
    riemann  -- exact solutions of the isothermal and barotropic Riemann problems
    conv     -- float64 reference of the 1D convolutional surrogate (forward,
                backward)
"""

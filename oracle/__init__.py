"""FP64 CPU oracle of the structured-grid weather step — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never imports, calls or links anything here, and this package never
imports the product path: the two share nothing but the seeded input arrays.

Every function is plain, slow and written to be checked against the paper by
eye: NumPy float64, periodic horizontal boundaries by ``np.roll`` (no halo
storage), one array expression per term of the definition, no fusion or
reordering.  Where the paper gives structure but not equations, the function
docstring states the reading it takes.

Modules
-------
params   constants of the readings (biharmonic strength, K_z closure, radiation)
dycore   3rd-order upwind face values, increment-form stage operator, RK3
physics  implicit vertical diffusion (Thomas) and the transmissivity k-scan
step     one full step = RK3 dycore followed by column physics
mass     compensated global mass sums
mlp      the surrogate network: forward, backward, Adam, with BF16 rounding
reduced  the paper's reduced weather application (7-point diffusion, column
         radiation and boundary heat exchange), to the last bit

Parity status: every function here is pinned by the CPU tests
(``tests/test_oracle_*.py``) against closed forms, invariants, a dense LAPACK
solve and brute force, except the surrogate's learned accuracy, which is
"parity unpinned" (there is no trained network in the paper to compare with).
"""

"""Plain FP64 CPU oracle for MRCM-OS right-preconditioned GMRES.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark use it.

The oracle is written from the paper (Zhou, Guiraldello, Pereira, Sousa,
"Accelerating GMRES with Matrix-Free Multiscale Robin Preconditioners"):

* ``discretization`` -- the fine system A p = b (Section 3, "New preconditioner
  with GMRES", first equation; model problem eqs. (1a)-(1d) of Section 2).
* ``partition``      -- non-overlapping subdomains, oversampled regions and
  smoothing patches (Section 2.1, the definitions of Omega_i, Gamma_i and
  hat-Omega_i, and the figure of the three scales).
* ``mrcm``           -- the MRCM-OS preconditioner T (Section 2.1 eqs.
  (11)-(14), the Robin condition and beta, the informed multiplier spaces and
  the oversampled problem; Section 3, the modified MRCM-O with source r and
  homogeneous boundary conditions).
* ``gmres``          -- right-preconditioned restarted GMRES (Algorithm 1).
* ``brute``          -- brute-force companions used only to pin the above on
  tiny grids.

Every function works in float64 with library primitives (sparse LU, dense
solves) as steps; there is no blocking, fusion or reordering beyond what the
definitions state.
"""

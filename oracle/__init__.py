"""Plain FP64 CPU oracle for the Newton-step linear solve of pressurized phase-field fracture.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or links this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` do.  It shares no code with the HIP path (no kernels, headers, helpers or
tables), and it is deliberately slow and direct: numpy/scipy element loops over Gauss
points, assembled with scipy.sparse, solved exactly (sparse LU or dense LU).

What it computes (Heister & Wick 2018, Section 2, Formulation 1 and Section 3):
  * Q1 finite elements on axis-aligned quads/hexes, 2-point Gauss per axis,
  * the residual of the displacement equation (E22ATW) and of the phase-field
    inequality (E33ATW),
  * their exact Jacobian blocks M_uu, M_phi_u, M_phi_phi (M_u_phi = 0),
  * the primal-dual active set for phi <= phi_old and the elimination of active rows,
  * the exact solution of the masked block lower-triangular system,
  * the Newton / active-set loop with line search (commented algorithm of Section 3),
  * the TCV and COD functionals and Sneddon's closed forms (Section 4).

Parity status per function is listed in each module header.
"""

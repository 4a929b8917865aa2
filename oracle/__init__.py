"""Plain FP64 CPU oracle of the implicit high-order Lagrangian hydrodynamics method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The GPU
library never calls it, and this package never calls the GPU library: the two share no
code, no tables and no constants.

The oracle follows the paper (Andrej et al., "Implicit Lagrangian Hydrodynamics with
High-Order Finite Elements") step by step, written plainly with dense per-element
matrices and NumPy/SciPy primitives:

* ``basis``   -- 1D Gauss-Lobatto-Legendre Lagrange (H1) and Bernstein (L2) bases,
                 Gauss-Legendre quadrature (Sec. 2.1, mixed Q_k Q_{k-1} spaces).
* ``mesh``    -- Cartesian box meshes, lexicographic H1 node grid, element maps.
* ``hydro``   -- quadrature data, mass matrices (eq. matrices), the force matrix
                 F_ij = int (sigma : grad w_i) phi_j (eq. matrices), the stage residual
                 (eq. nonlinear_system), EOS with energy regularization
                 (eq. energy_regularization), smoothed viscosity (eqs. visc_stress,
                 visc_mu_imp .. visc_imp_scale), energy and diagnostics.
* ``krylov``  -- complex-step Jacobian actions (eq. pa_jac_action realised as an exact
                 derivative), Jacobi-PCG, restarted flexible GMRES, Newton with the
                 detJ line search (Sec. 3.5) and the implicit midpoint step.
* ``mlp``     -- reference MLP (BF16-rounded weights/activations, FP32 accumulation)
                 for the learned Newton initial guess.

Functions whose result has no independent pin say "parity unpinned" in their docstring.
"""

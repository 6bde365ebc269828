"""CPU oracle for the PHS + polynomial RBF-FD hot path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product library
never does. It is a plain, slow, FP64 restatement of what the method computes:

* ``stencils.knn``       -- n nearest nodes per centre, key (d^2, j)
                            (Section 6: n = 37 stencils; Appendix A shells)
* ``weights.stencil_weights`` -- one saddle-point solve per stencil
                            (Section 3, Eq. weights; Section 5.3, Eq. eqn:laplacian)
* ``rhs.advection_rhs``  -- flux-form scalar transport (Section 6.1)
* ``rhs.ghost_closure``  -- ghost values from W_G u_G = -(W_I u_I + W_B u_B)
                            (Section 5.2, Eq. bcEqn; BCs of Section 6.4)
* ``rhs.ns_rhs``         -- Eqs. uEq, wEq, thetaEq, piEq + hyperviscosity
* ``timestep``           -- classical RK4 (Section 6) and a 3-stage RK
* ``diagnostics``        -- extrema, front location, relative l2 error

It shares no code with the HIP path; both read their inputs from the
``workloads`` package, which holds no method arithmetic.
"""

from .stencils import knn, min_image
from .weights import (
    DX, DZ, LAP, HYPERLAP, DZZ, DXX, poly_exponents, phs_apply, poly_apply,
    stencil_weights, all_weights, op_order,
)
from .rhs import apply_dm, dm_matrix, advection_rhs, AdvectionModel, ghost_matrices, ghost_closure, ns_rhs, ns_tendency, NSModel, WallRows
from .timestep import rk4_step, wsrk3_step, integrate
from .diagnostics import rel_l2, front_location, extrema, translating_fronts, bubble_height

"""Seeded synthetic inputs shaped like the paper's workloads.

This package is shared by the CPU oracle and the HIP path, so it holds no
RBF-FD arithmetic at all: only node coordinates (Section 5.1 layouts and the
Section 6 test domains), node kinds, seeded jitter, initial/synthetic field
values and the physical constants of the test cases (Section 6.2, 6.4).
"""

from .nodes import NodeSet, unit_square_cartesian, channel, straka_nodes, jittered_square, box
from .fields import (
    NS_CONSTANTS, cosine_bell, swirl_velocity, straka_theta, smooth_ns_state,
    ensemble_amplitudes, bubble_state,
)
from .configs import (
    advection_config, density_current_config, weights_config, scale_config, translating_config,
    closure_config, bubble_config,
)

"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds no arithmetic of the solver: it only describes meshes
(connectivity tables, cell sizes), the linearisation state (reference
profiles of potential temperature and Exner pressure, density) and the
random right-hand sides.  Both the CPU oracle and the HIP library consume
what it produces; neither imports the other.
"""

from .box import BoxProblem, make_box, make_rhs, make_rhs_p1, config_box  # noqa: F401
from .sphere import SphereProblem, make_sphere, make_rhs_sphere, config_sphere  # noqa: F401,E402

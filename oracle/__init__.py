"""FP64 CPU oracle of the Swarm-Gen safety filter (Appendix, "Custom SF optimizer").

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call this
package: only the tests, the smoke check of the entry module and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library.
"""
from .sf_oracle import (  # noqa: F401
    bernstein,
    basis_matrices,
    pair_incidence,
    OracleSystem,
    build_system,
    project_collision,
    project_ball,
    project_workspace,
    sf_project,
    feasibility,
    qp_equality,
    to_paper_order,
    from_paper_order,
)

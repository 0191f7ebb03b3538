"""FP64 CPU oracle for DID (distributed incremental block coordinate descent for NMF).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP engine under
``paper_1802_08938_amd/``; the only thing both sides consume is the seeded input
generators in ``workloads/``, which hold none of the method's arithmetic.

Modules
-------
``did``     the method itself, step by step in the paper's order (Alg. 3).
``bcd``     the textbook sequential block coordinate descent that DID reorganises
            (eqs. sol:c_ij and sol:b_i 2 evaluated from scratch), plus the DBCD
            variant of Alg. 2.  Used as an independent cross-check of ``did``.
"""

from .did import (  # noqa: F401
    project,
    objective,
    residual,
    column_blocks,
    c_half,
    messages,
    b_half,
    did_iteration,
    did_run,
    iterations_to_tolerance,
)
from .bcd import naive_bcd_iteration, naive_bcd_run, dbcd_iteration  # noqa: F401

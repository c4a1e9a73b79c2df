"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library neither imports nor
links it, and the two share no code.
"""

from .oracle import (  # noqa: F401
    OracleTree,
    build_library,
    eigh3,
    octant_init,
    em_partition,
    build_tree,
    build_root,
    build_level,
    estep,
    estep_flat,
    normal_equations,
    solve_update,
    register,
    register_flat,
    estep_soft,
    register_soft,
    compose_chain,
    level_offset,
    level_nodes,
)
from . import warm  # noqa: F401

"""CPU oracle for round-synchronous 2D constrained Delaunay refinement.

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU path is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU
baseline may import it; the product package never does.
"""
from .api import (  # noqa: F401
    OracleError,
    OracleMesh,
    build_cdt,
    refine,
    ruppert,
    mesh_from_arrays,
    orient2d,
    incircle,
    indiametral,
    encroaches,
    incircle_sos,
    perm32,
    exact_counts,
    load,
)

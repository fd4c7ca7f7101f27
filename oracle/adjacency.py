"""ORACLE -- test infrastructure only.

The adjacency a smoothing pass takes as input, built from a bare triangle
list the way the paper describes it, in plain Python loops (small meshes
only):

* Finding of neighbours (Sec. 3.3.2): the triangles are visited in index
  order; a triangle (v1, v2, v3) records v2 and v3 as neighbours of v1, v1
  and v3 as neighbours of v2, and v1 and v2 as neighbours of v3, in that
  order.  A node's row keeps each neighbour once, where it first appeared.
  Each triangle is incident to its three vertices; a node's incident
  triangles are listed in index order.
* Determining of constraints (Sec. 3.3.3): a node is interior when every one
  of its neighbours was recorded exactly twice (every edge at the node lies
  in two triangles); otherwise, and for a node in no triangle, it is a
  boundary node.

Shares no code with the GPU library or with the mesh generators.
"""
from __future__ import annotations

import numpy as np


def adjacency(n_nodes: int, tris):
    """(nbr_ptr, nbr_idx, tri_ptr, tri_idx, boundary) as int32 / uint8 arrays."""
    tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    rows = [[] for _ in range(n_nodes)]
    seen = [dict() for _ in range(n_nodes)]
    incident = [[] for _ in range(n_nodes)]
    for t in range(tris.shape[0]):
        v1, v2, v3 = (int(v) for v in tris[t])
        for owner, others in ((v1, (v2, v3)), (v2, (v1, v3)), (v3, (v1, v2))):
            incident[owner].append(t)
            for u in others:
                if u in seen[owner]:
                    seen[owner][u] += 1
                else:
                    seen[owner][u] = 1
                    rows[owner].append(u)
    nbr_ptr = np.zeros(n_nodes + 1, np.int32)
    tri_ptr = np.zeros(n_nodes + 1, np.int32)
    for v in range(n_nodes):
        nbr_ptr[v + 1] = nbr_ptr[v] + len(rows[v])
        tri_ptr[v + 1] = tri_ptr[v] + len(incident[v])
    nbr_idx = np.array([u for r in rows for u in r], dtype=np.int32)
    tri_idx = np.array([t for r in incident for t in r], dtype=np.int32)
    boundary = np.array([0 if rows[v] and all(c == 2 for c in seen[v].values()) else 1 for v in range(n_nodes)],
                        dtype=np.uint8)
    return nbr_ptr, nbr_idx, tri_ptr, tri_idx, boundary

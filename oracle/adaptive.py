"""Adaptive quadtree / octree meshes with hanging nodes for the oracle (Section 3: adaptive
Q1^c meshes; conformity by hanging-node constraints).

Refinement rule (the workload's, shared with the library by definition, implemented here
independently): starting from n^d equal cells on [lo, hi]^d, a cell is split into 2^d
children while its level is below `levels` and the distance from its box to the crack
(2d: the segment |x - c_x| <= l on y = c_y; 3d: the disk of radius l in z = c_z) is at most
`radius`.  Afterwards cells are split until neighbouring cells (sharing any point) differ by
at most one level (2:1 balance).

Hanging nodes: a vertex of a finer cell that lies at the midpoint of an edge of a coarser
cell takes half of each edge end; one at the centre of a coarser cell's face (3d) takes a
quarter of each face corner.  The conformity map C (n_nodes x n_free) holds these weights.

Pinned by tests/test_oracle_adaptive.py: the cells tile the domain, 2:1 balance, linear
fields are reproduced by C, the patch test (zero interior residual for a linear displacement)
on the condensed system, finite differences of the condensed residual against the condensed
Jacobian, and the lumped mass summing to |B|.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


def _box_distance(dim, a, b, center, l):
    if dim == 2:
        dx = max(0.0, (center[0] - l) - b[0], a[0] - (center[0] + l))
        dy = max(0.0, center[1] - b[1], a[1] - center[1])
        return np.hypot(dx, dy)
    px = min(max(center[0], a[0]), b[0])
    py = min(max(center[1], a[1]), b[1])
    dxy = max(0.0, np.hypot(px - center[0], py - center[1]) - l)
    dz = max(0.0, center[2] - b[2], a[2] - center[2])
    return np.hypot(dxy, dz)


def adaptive(dim, lo, hi, n, levels, radius, center, half_len):
    S = 1 << levels                      # lattice units per base cell
    h_min = (hi - lo) / n / S
    ext = n * S

    # leaves as {(level, origin tuple)}
    leaves = set()
    stack = [(0, tuple(int(i) * S for i in idx)) for idx in itertools.product(range(n), repeat=dim)]
    while stack:
        lev, o = stack.pop()
        s = S >> lev
        a = [lo + o[k] * h_min for k in range(dim)]
        b = [lo + (o[k] + s) * h_min for k in range(dim)]
        if lev < levels and _box_distance(dim, a, b, center, half_len) <= radius:
            for ch in itertools.product((0, 1), repeat=dim):
                stack.append((lev + 1, tuple(o[k] + ch[k] * s // 2 for k in range(dim))))
        else:
            leaves.add((lev, o))
    return mesh_from_leaves(dim, lo, hi, h_min, S, ext, balance(dim, S, ext, leaves))


def balance(dim, S, ext, leaves):
    """Splits leaves {(level, origin)} until cells sharing a point differ by at most one level."""
    leaves = set(leaves)

    def leaf_at(point, max_level):
        for lev in range(max_level + 1):
            s = S >> lev
            o = tuple((point[k] // s) * s for k in range(dim))
            if (lev, o) in leaves:
                return lev, o
        return None

    changed = True
    while changed:
        changed = False
        split = set()
        for lev, o in leaves:
            if lev < 2:
                continue
            s = S >> lev
            for off in itertools.product((-1, 0, 1), repeat=dim):
                if not any(off):
                    continue
                q = tuple(o[k] + off[k] * s + (s // 2 if s > 1 else 0) for k in range(dim))
                if any(q[k] < 0 or q[k] >= ext for k in range(dim)):
                    continue
                found = leaf_at(q, lev)
                if found is not None and found[0] < lev - 1:
                    split.add(found)
        for lev, o in split:
            if (lev, o) in leaves:
                leaves.remove((lev, o))
                s = S >> lev
                for ch in itertools.product((0, 1), repeat=dim):
                    leaves.add((lev + 1, tuple(o[k] + ch[k] * s // 2 for k in range(dim))))
                changed = True
    return leaves


def mesh_from_leaves(dim, lo, hi, h_min, S, ext, leaves):
    """Nodes, cells, hanging constraints and Dirichlet flags of a balanced leaf set."""
    cells_l = sorted(leaves, key=lambda t: (tuple(reversed(t[1])), t[0]))
    nv = 1 << dim
    bits = np.array([[(a >> k) & 1 for k in range(dim)] for a in range(nv)])
    P = ext + 1

    def key(q):
        return sum(int(q[k]) * P ** k for k in range(dim))

    vert_keys = []
    for lev, o in cells_l:
        s = S >> lev
        for a in range(nv):
            vert_keys.append(key([o[k] + bits[a, k] * s for k in range(dim)]))
    uk = np.unique(np.array(vert_keys, dtype=np.int64))
    index = {int(k): i for i, k in enumerate(uk)}
    lattice = np.stack([(uk // P ** k) % P for k in range(dim)], axis=1)
    coords = lo + lattice * h_min
    cells = np.array(vert_keys, dtype=np.int64).reshape(-1, nv)
    cells = np.vectorize(lambda k: index[int(k)])(cells)
    cell_lo = np.array([[lo + o[k] * h_min for k in range(dim)] for _, o in cells_l])
    cell_h = np.array([(S >> lev) * h_min for lev, _ in cells_l])

    # hanging nodes
    hang = {}
    for c, (lev, o) in enumerate(cells_l):
        s = S >> lev
        if s < 2:
            continue
        cv = cells[c]
        for a in range(nv):
            for k in range(dim):
                if bits[a, k]:
                    continue
                b = a | (1 << k)
                q = [o[t] + bits[a, t] * s for t in range(dim)]
                q[k] += s // 2
                n_id = index.get(key(q))
                if n_id is not None and n_id not in hang:
                    hang[n_id] = [(cv[a], 0.5), (cv[b], 0.5)]
        if dim == 3:
            for k in range(3):
                for side in (0, 1):
                    q = [o[t] + s // 2 for t in range(3)]
                    q[k] = o[k] + side * s
                    n_id = index.get(key(q))
                    if n_id is not None and n_id not in hang:
                        hang[n_id] = [(cv[a], 0.25) for a in range(nv) if bits[a, k] == side]
    # masters that are themselves hanging are substituted
    for n_id in list(hang):
        for _ in range(8):
            if not any(m in hang for m, _ in hang[n_id]):
                break
            new = {}
            for m, w in hang[n_id]:
                if m in hang:
                    for m2, w2 in hang[m]:
                        new[m2] = new.get(m2, 0.0) + w * w2
                else:
                    new[m] = new.get(m, 0.0) + w
            hang[n_id] = sorted(new.items())

    n_nodes = len(uk)
    is_free = np.ones(n_nodes, dtype=bool)
    is_free[list(hang.keys())] = False
    free = np.nonzero(is_free)[0]
    free_of = -np.ones(n_nodes, dtype=np.int64)
    free_of[free] = np.arange(len(free))
    rows, cols, vals = [], [], []
    for nd in range(n_nodes):
        if is_free[nd]:
            rows.append(nd); cols.append(free_of[nd]); vals.append(1.0)
        else:
            for m, w in hang[nd]:
                rows.append(nd); cols.append(free_of[m]); vals.append(w)
    C = sp.csr_matrix((vals, (rows, cols)), shape=(n_nodes, len(free)))
    dirichlet = np.any((lattice == 0) | (lattice == ext), axis=1)
    m = Mesh(dim, coords, lattice, cells, cell_lo, cell_h, dirichlet, C, free, lo, hi)
    m.S = S
    m.leaves = cells_l
    return m

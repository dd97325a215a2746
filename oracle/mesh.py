"""Oracle meshes: axis-aligned quads (2d) / hexes (3d) on B = [lo, hi]^d.

Section 3: Q1^c on quadrilaterals / hexahedra; Section 2: homogeneous Dirichlet data for
the displacement on the whole outer boundary, no boundary condition on phi (W = H^1(B)).

A mesh is described by
  coords[n_nodes, d], lattice[n_nodes, d] (integer coordinates on the finest lattice),
  cells[n_cells, 2^d] (vertex node ids, vertex a at lower corner + bits of a),
  cell_lo[n_cells, d], cell_h[n_cells],
  dirichlet[n_nodes] (node on the outer boundary),
  C (scipy CSR, n_nodes x n_free): nodal values = C @ free values, the hanging-node
  conformity map (identity on uniform meshes; edge midpoints 1/2 + 1/2, face centres
  1/4 each, in the adaptive mesh of oracle.adaptive),
  free[n_free]: node id of each free (non-hanging) node, in solve order.

Uniform meshes number nodes lexicographically (x fastest), cells likewise.

Pinned by tests/test_oracle_basics.py (test_table1_dof_counts: the Table 1 DoF counts
3 (2^(k+3)+1)^2; test_uniform_mesh_geometry: node and cell counts, vertex coordinates
consistent with cell corners).
"""
import numpy as np
import scipy.sparse as sp


class Mesh:
    def __init__(self, dim, coords, lattice, cells, cell_lo, cell_h, dirichlet, C, free, lo, hi):
        self.dim = dim
        self.coords = coords
        self.lattice = lattice
        self.cells = cells
        self.cell_lo = cell_lo
        self.cell_h = cell_h
        self.dirichlet = dirichlet
        self.C = C
        self.free = free
        self.lo = lo
        self.hi = hi

    @property
    def n_nodes(self):
        return self.coords.shape[0]

    @property
    def n_cells(self):
        return self.cells.shape[0]

    @property
    def n_free(self):
        return self.free.shape[0]

    @property
    def n_all(self):
        """All nodal DoFs, the convention of Table 1: (d + 1) n_nodes."""
        return (self.dim + 1) * self.n_nodes

    @property
    def n_solve(self):
        """Rows of the solved system: (d + 1) per free node (Dirichlet rows kept)."""
        return (self.dim + 1) * self.n_free

    @property
    def h_min(self):
        return float(self.cell_h.min())


def uniform(dim, lo, hi, n):
    """n^d equal cells on [lo, hi]^d."""
    h = (hi - lo) / n
    ax = np.arange(n + 1)
    if dim == 2:
        J, I = np.meshgrid(ax, ax, indexing="ij")
        lattice = np.stack([I.ravel(), J.ravel()], axis=1)
    else:
        K, J, I = np.meshgrid(ax, ax, ax, indexing="ij")
        lattice = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    coords = lo + lattice * h
    stride = np.array([(n + 1) ** k for k in range(dim)])
    cax = np.arange(n)
    if dim == 2:
        J, I = np.meshgrid(cax, cax, indexing="ij")
        clat = np.stack([I.ravel(), J.ravel()], axis=1)
    else:
        K, J, I = np.meshgrid(cax, cax, cax, indexing="ij")
        clat = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    nv = 1 << dim
    bits = np.array([[(a >> k) & 1 for k in range(dim)] for a in range(nv)])
    cells = ((clat[:, None, :] + bits[None, :, :]) * stride).sum(axis=2)
    cell_lo = lo + clat * h
    cell_h = np.full(clat.shape[0], h)
    dirichlet = np.any((lattice == 0) | (lattice == n), axis=1)
    n_nodes = coords.shape[0]
    C = sp.identity(n_nodes, format="csr")
    free = np.arange(n_nodes)
    m = Mesh(dim, coords, lattice, cells, cell_lo, cell_h, dirichlet, C, free, lo, hi)
    m.S = 1                                   # lattice units per base cell (no refinement)
    m.leaves = [(0, tuple(int(v) for v in o)) for o in clat]
    return m

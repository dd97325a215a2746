"""Mesh refinement between loading steps, solution transfer and crack-region marks.

TEST INFRASTRUCTURE ONLY (see the package header).

Section 3 refines the mesh so that eps = 2h holds in the crack region, and by a gradient-jump
indicator of the displacements.  Between loading steps:
  * marks: a cell is marked when its edge exceeds h_target and phi is below phi_max at one of
    its vertices (the crack region; phi_max and h_target are the caller's, e.g. eps / 2);
  * refinement: every marked leaf is split into 2^d children, then the 2:1 balance of the
    adaptive meshes is restored (oracle/adaptive.py);
  * transfer: every node of the new mesh takes the value of the old Q1 function at its
    position.  The new space contains the old one, so the function is unchanged;
  * gradient-jump indicator (Kelly type): eta_K^2 = h_K / 24 * sum over the faces F of K of
    the integral over F of |[du/dn]|^2 summed over the components, the jump taken across F,
    zero on the boundary.  Reading: the paper names the estimator only; h_K is the cell edge
    and the weight 1/24 is the customary one (a constant factor does not change which cells
    rank highest).  Each face is integrated on its intersection with every neighbour across
    it, by the 2-point Gauss rule per tangential axis, exact for the squared jump of Q1
    gradients.
Reading: marks use nodal phi (hanging vertices interpolated), a vertex test rather than a
cell average, since the band of a sharp initial crack is a single node layer on coarse cells.

Pinned by tests/test_oracle_refine.py: splitting every cell of a uniform mesh gives the
uniform mesh of half the edge; marked cells end up split, the result tiles the domain and is
2:1 balanced; the transferred field equals the old function at random points of every cell
(brute-force cell search) and reproduces bilinear fields exactly; marks against a direct scan;
the indicator vanishes for globally linear displacements (hanging nodes included) and equals
the closed form h^2/6 (2d) next to a grid line where du_0/dx_0 jumps by 2.
"""
import itertools

import numpy as np

from .adaptive import balance, mesh_from_leaves


def leaves_of(m):
    """(level, origin) of every cell, in cell order, lattice units of m."""
    return list(m.leaves)


def refine(m, flags):
    """The mesh with every flagged cell split, then 2:1 balanced."""
    dim = m.dim
    S = m.S
    L = int(round(np.log2(S)))
    lv = leaves_of(m)
    grow = any(bool(flags[c]) and lev == L for c, (lev, _) in enumerate(lv))
    f = 2 if grow else 1
    S2 = S * f
    n_base = int(m.lattice.max()) // S          # base cells per axis
    ext2 = n_base * S2
    new = set()
    for c, (lev, o) in enumerate(lv):
        o2 = tuple(x * f for x in o)
        if flags[c]:
            s = S2 >> lev
            for ch in itertools.product((0, 1), repeat=dim):
                new.add((lev + 1, tuple(o2[k] + ch[k] * (s // 2) for k in range(dim))))
        else:
            new.add((lev, o2))
    unit = (m.hi - m.lo) / n_base / S2          # lattice unit: base edge / S2
    return mesh_from_leaves(dim, m.lo, m.hi, unit, S2, ext2, balance(dim, S2, ext2, new))


def _locate(m, x):
    """Index of a cell of m that contains point x (closed boxes), by a scan of all cells."""
    lo = m.cell_lo
    hi = m.cell_lo + m.cell_h[:, None]
    tol = 1e-12 * (m.hi - m.lo)
    inside = np.all((x[None, :] >= lo - tol) & (x[None, :] <= hi + tol), axis=1)
    return int(np.nonzero(inside)[0][0])


def evaluate(m, values, x):
    """The Q1 function of m with nodal values `values` ([n_nodes] or [n_nodes, k]; hanging
    values from the constraints) at point x."""
    dim = m.dim
    v = np.asarray(values, dtype=np.float64)
    full = m.C @ v[m.free]
    c = _locate(m, x)
    xi = (x - m.cell_lo[c]) / m.cell_h[c]
    out = 0.0
    for a in range(1 << dim):
        w = 1.0
        for k in range(dim):
            w *= xi[k] if (a >> k) & 1 else 1.0 - xi[k]
        out = out + w * full[m.cells[c, a]]
    return out


def transfer(old, new, values):
    """Nodal values on `new` of the old Q1 function."""
    return np.array([evaluate(old, values, new.coords[n]) for n in range(new.n_nodes)])


def mark_crack(m, phi, phi_max, h_target):
    """uint8 marks per cell: edge > h_target and phi < phi_max at a vertex."""
    full = m.C @ np.asarray(phi, dtype=np.float64)[m.free]
    low = full[m.cells].min(axis=1) < phi_max
    return ((m.cell_h > h_target) & low).astype(np.uint8)


def _grad(m, full, c, x):
    """Gradient [comp, k] at point x of the Q1 field `full` ([n_nodes, ncomp]) on cell c."""
    dim = m.dim
    h = m.cell_h[c]
    xi = (x - m.cell_lo[c]) / h
    g = np.zeros((full.shape[1], dim))
    for a in range(1 << dim):
        for k in range(dim):
            w = 1.0 if (a >> k) & 1 else -1.0
            for t in range(dim):
                if t != k:
                    w *= xi[t] if (a >> t) & 1 else 1.0 - xi[t]
            g[:, k] += w / h * full[m.cells[c, a]]
    return g


def kelly(m, u):
    """eta^2 per cell for the displacement u [n_nodes, dim] (hanging values from C)."""
    dim = m.dim
    full = m.C @ np.asarray(u, dtype=np.float64).reshape(m.n_nodes, -1)[m.free]
    lo = m.cell_lo
    hi = m.cell_lo + m.cell_h[:, None]
    tol = 1e-12 * (m.hi - m.lo)
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    eta2 = np.zeros(m.n_cells)
    for c in range(m.n_cells):
        acc = 0.0
        for k in range(dim):
            for side in (0, 1):
                plane = lo[c, k] + side * m.cell_h[c]
                other = (np.abs(lo[:, k] - plane) <= tol) if side else (np.abs(hi[:, k] - plane) <= tol)
                tang = [t for t in range(dim) if t != k]
                for t in tang:
                    other &= (np.minimum(hi[:, t], hi[c, t]) - np.maximum(lo[:, t], lo[c, t])) > tol
                for n in np.nonzero(other)[0]:
                    a = [max(lo[c, t], lo[n, t]) for t in tang]
                    b = [min(hi[c, t], hi[n, t]) for t in tang]
                    w = np.prod([(bb - aa) / 2.0 for aa, bb in zip(a, b)])
                    for q in np.ndindex(*([2] * (dim - 1))):
                        x = np.empty(dim)
                        x[k] = plane
                        for i, t in enumerate(tang):
                            x[t] = a[i] + (b[i] - a[i]) * gp[q[i]]
                        jump = _grad(m, full, c, x)[:, k] - _grad(m, full, n, x)[:, k]
                        acc += w * float(jump @ jump)
        eta2[c] = m.cell_h[c] / 24.0 * acc
    return eta2

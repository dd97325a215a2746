"""TCV and COD functionals (Section 4) and Sneddon's closed forms.

TCV_h = integral over B of u . grad phi, by the Q1 Gauss rule on every cell (the paper
writes the domain as Omega; reading: all of B, since grad phi vanishes inside the fully
broken band).

COD_h(x0) = 1/2 integral of u . grad phi along the line through x0 normal to the crack
(the last axis), with the 1d 2-point Gauss rule on every cell the line crosses (half-open
cells [lo, lo + h) along the other axes).  The paper gives only the closed form of the
crack opening displacement; the factor 1/2 maps the full opening jump, which the line
integral measures, to the one-face displacement u_n of the closed form, consistent with
TCV = integral of 2 u_n.

Closed forms (Section 4, Sneddon):
  2d: TCV = 2 pi p l0^2 (1-nu^2)/E,  u_n(x) = 2 p l0 (1-nu^2)/E sqrt(1 - (x/l0)^2)
  3d: TCV = 16 p l0^3 (1-nu^2)/(3E), u_n(rho) = (4/pi) p l0 (1-nu^2)/E sqrt(1 - (rho/l0)^2)

Pinned by tests/test_oracle_basics.py: exact values for Q1-representable fields
(u = e_0, phi linear in x_0 gives TCV = |B| / (hi - lo); COD of u = e_last, phi linear
in the last axis), the paper's printed value 6.0319E-03 of the 2d closed form, the
integral of 2 u_n reproducing TCV (2d and 3d).
"""
import numpy as np

from . import q1


def tcv(mesh, u, phi):
    d = mesh.dim
    Nr, dNr, _ = q1.reference(d)
    h = mesh.cell_h
    ue = u[mesh.cells]                                  # [e, a, c]
    pe = phi[mesh.cells]
    uq = np.einsum("eac,qa->eqc", ue, Nr)
    gp = np.einsum("ea,qak->eqk", pe, dNr) * (2.0 / h)[:, None, None]
    W = (0.5 * h) ** d
    return float((np.einsum("eqc,eqc->e", uq, gp) * W).sum())


def cod(mesh, u, phi, x0):
    """x0[d-1]: the position of the line along the first d-1 axes."""
    d = mesh.dim
    x0 = np.atleast_1d(np.asarray(x0, dtype=np.float64))
    lo = mesh.cell_lo
    h = mesh.cell_h
    hit = np.ones(mesh.n_cells, dtype=bool)
    for k in range(d - 1):
        hit &= (lo[:, k] <= x0[k]) & (x0[k] < lo[:, k] + h)
    idx = np.nonzero(hit)[0]
    total = 0.0
    gq = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    for e in idx:
        he = h[e]
        xi = np.empty((2, d))
        for k in range(d - 1):
            xi[:, k] = 2.0 * (x0[k] - lo[e, k]) / he - 1.0
        xi[:, d - 1] = gq
        N = q1.shape(d, xi)
        dN = q1.shape_grad(d, xi) * (2.0 / he)
        ue = u[mesh.cells[e]]
        pe = phi[mesh.cells[e]]
        uq = N @ ue
        gp = np.einsum("a,qak->qk", pe, dN)
        total += 0.5 * he * np.einsum("qc,qc->", uq, gp)
    return 0.5 * total


def sneddon_tcv(dim, p, l0, E, nu):
    if dim == 2:
        return 2.0 * np.pi * p * l0 ** 2 * (1.0 - nu ** 2) / E
    return 16.0 * p * l0 ** 3 * (1.0 - nu ** 2) / (3.0 * E)


def sneddon_cod(dim, p, l0, E, nu, rho):
    c = 2.0 if dim == 2 else 4.0 / np.pi
    rho = np.asarray(rho, dtype=np.float64)
    return c * p * l0 * (1.0 - nu ** 2) / E * np.sqrt(np.maximum(0.0, 1.0 - (rho / l0) ** 2))

"""Residual and Jacobian of Formulation 1 (Section 2) on Q1 elements, FP64.

State: u[n_nodes, d], phi[n_nodes], phi_tilde[n_nodes] on all mesh nodes (hanging nodes
carry the interpolated value C @ free).  At each Gauss point:
    g     = (1 - kappa) phi_tilde^2 + kappa                       (stiffness degradation)
    e(u)  = (grad u + grad u^T) / 2,  sigma = 2 mu e + lambda tr(e) I   (linear elastic law)
    s     = sigma : e,  theta = div u = tr e.

Residual, tested with every basis function (equations E22ATW and E33ATW):
    R_u[a, c]  = sum_q W ( g sigma[c, k] dN_a[k] + phi_tilde^2 p dN_a[c] )
    R_phi[a]   = sum_q W ( (1-kappa) phi s N_a + 2 p phi theta N_a
                           - (G_c/eps) (1 - phi) N_a + G_c eps grad phi . grad N_a )
Reading (phi or phi_tilde in the pressure term of E22ATW): the paper writes phi^2 in
E22ATW but states that M_u_phi vanishes because of phi_tilde (Section 3, Linear
iterative solution).  Only phi_tilde^2 in both u-equation terms gives M_u_phi = 0, so the
oracle uses phi_tilde^2 there.

Jacobian (exact derivative of the residual; Section 3 lists the blocks):
    M_uu[(a,c),(b,d)] = sum_q W g ( mu (delta_cd dN_b.dN_a + dN_b[c] dN_a[d]) + lambda dN_b[d] dN_a[c] )
    M_phiu[a,(b,d)]   = sum_q W ( 2 (1-kappa) phi sigma[d,k] dN_b[k] + 2 p phi dN_b[d] ) N_a
    M_phiphi[a,b]     = sum_q W ( ((1-kappa) s + 2 p theta + G_c/eps) N_b N_a + G_c eps dN_b.dN_a )
Readings: the extra undegraded "+ (sigma(chi_j), e(chi_i))" printed in M_uu is not a
derivative of E22ATW and is dropped; the undefined alpha in M_phiu / M_phiphi is taken as
0, which gives the +2p of the phi inequality.  The finite-difference test pins all three.

Solve ordering (Section 3, block basis): u block node-major over the free nodes
(index f*d + c), then the phi block (index d*n_free + f).

Pinned by tests/test_oracle_fem.py: R(0, phi=1) = 0 in the interior; patch test (linear u
gives zero interior R_u); energy identity u.R_u = |B| sigma(e):e for homogeneous strain;
closed-form sums of R_phi for constant phi and homogeneous strain; discrete Laplacian of
x^2; central finite differences of R against every Jacobian block (and zero u-phi block);
rigid-body modes in the kernel of the unconstrained elasticity stiffness.
"""
import numpy as np
import scipy.sparse as sp

from . import q1


def _cell_data(mesh, cells_idx):
    Nr, dNr, w = q1.reference(mesh.dim)
    h = mesh.cell_h[cells_idx]
    scale = (2.0 / h)[:, None, None, None]            # d xi / d x
    dN = dNr[None, :, :, :] * scale                     # [e, q, a, k]
    W = (0.5 * h) ** mesh.dim                          # w_q |J|, w_q = 1
    return Nr, dN, W


def qp_fields(mesh, prm, u, phi, phi_tilde, cells_idx=None):
    """Per-cell, per-Gauss-point fields (equations E22ATW / E33ATW ingredients)."""
    if cells_idx is None:
        cells_idx = np.arange(mesh.n_cells)
    d = mesh.dim
    conn = mesh.cells[cells_idx]
    Nr, dN, W = _cell_data(mesh, cells_idx)
    ue = u[conn]                                         # [e, a, c]
    pe = phi[conn]
    pte = phi_tilde[conn]
    gu = np.einsum("eac,eqak->eqck", ue, dN)            # grad u [e, q, c, k]
    eps_t = 0.5 * (gu + np.swapaxes(gu, 2, 3))
    tr = np.trace(eps_t, axis1=2, axis2=3)
    sig = 2.0 * prm.mu * eps_t + prm.lam * tr[:, :, None, None] * np.eye(d)[None, None]
    s = np.einsum("eqck,eqck->eq", sig, eps_t)
    ph = pe @ Nr.T                                       # [e, q]
    gph = np.einsum("ea,eqak->eqk", pe, dN)
    pt = pte @ Nr.T
    g = (1.0 - prm.kappa) * pt ** 2 + prm.kappa
    return dict(conn=conn, N=Nr, dN=dN, W=W, gu=gu, sig=sig, s=s, theta=tr,
                phi=ph, gphi=gph, pt=pt, g=g)


def residual_all(mesh, prm, u, phi, phi_tilde, cells_idx=None):
    """Uncondensed residual on all nodes: R_u[n_nodes, d], R_phi[n_nodes], and the
    row sums of the phi mass matrix (lumped mass) mass[n_nodes]."""
    f = qp_fields(mesh, prm, u, phi, phi_tilde, cells_idx)
    d = mesh.dim
    W = f["W"][:, None]
    N, dN = f["N"], f["dN"]
    # E22ATW tested with w = N_a e_c
    t1 = np.einsum("eq,eqck,eqak->eac", f["g"], f["sig"], dN)
    t2 = np.einsum("eq,eqac->eac", f["pt"] ** 2 * prm.p, dN)
    Ru_loc = (t1 + t2) * W[:, :, None]
    # E33ATW tested with psi - phi = N_a
    react = ((1.0 - prm.kappa) * f["phi"] * f["s"] + 2.0 * prm.p * f["phi"] * f["theta"]
             - (prm.Gc / prm.eps) * (1.0 - f["phi"]))
    Rp_loc = (np.einsum("eq,qa->ea", react, N)
              + prm.Gc * prm.eps * np.einsum("eqk,eqak->ea", f["gphi"], dN)) * W
    m_loc = np.broadcast_to(N.sum(axis=0)[None, :], Rp_loc.shape) * W
    conn = f["conn"].ravel()
    n = mesh.n_nodes
    Ru = np.zeros((n, d))
    for c in range(d):
        Ru[:, c] = np.bincount(conn, weights=Ru_loc[:, :, c].ravel(), minlength=n)
    Rp = np.bincount(conn, weights=Rp_loc.ravel(), minlength=n)
    m = np.bincount(conn, weights=m_loc.ravel(), minlength=n)
    return Ru, Rp, m


def block_C(mesh):
    """Conformity map from solve-order unknowns to all-node unknowns.

    Rows: all-node unknowns (u: node*d + c, then phi: d*n_nodes + node).
    Columns: solve order (u: f*d + c, then phi: d*n_free + f)."""
    d = mesh.dim
    C = mesh.C.tocoo()
    rows, cols, vals = [], [], []
    for c in range(d):
        rows.append(C.row * d + c)
        cols.append(C.col * d + c)
        vals.append(C.data)
    rows.append(d * mesh.n_nodes + C.row)
    cols.append(d * mesh.n_free + C.col)
    vals.append(C.data)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=((d + 1) * mesh.n_nodes, (d + 1) * mesh.n_free))


def residual(mesh, prm, u, phi, phi_tilde):
    """Condensed residual in solve order, and the condensed lumped phi mass B[n_free].

    Condensation (hanging nodes): R_tilde = C^T R (each free basis function is the
    conforming combination of the nodal Q1 functions)."""
    Ru, Rp, m = residual_all(mesh, prm, u, phi, phi_tilde)
    d = mesh.dim
    R_all = np.concatenate([Ru.ravel(), Rp])
    R = block_C(mesh).T @ R_all
    B = mesh.C.T @ m
    return R, B


def element_matrices(mesh, prm, u, phi, phi_tilde, cells_idx=None):
    """K_uu[e,a,c,b,d], K_phiu[e,a,b,d], K_phiphi[e,a,b] (Section 3 block entries)."""
    f = qp_fields(mesh, prm, u, phi, phi_tilde, cells_idx)
    d = mesh.dim
    W = f["W"]
    N, dN = f["N"], f["dN"]
    g = f["g"]
    I = np.eye(d)
    lap = np.einsum("eqbk,eqak->eqab", dN, dN)
    Kuu = prm.mu * np.einsum("eq,cd,eqab->eacbd", g, I, lap)
    Kuu += prm.mu * np.einsum("eq,eqbc,eqad->eacbd", g, dN, dN)
    Kuu += prm.lam * np.einsum("eq,eqbd,eqac->eacbd", g, dN, dN)
    Kuu *= W[:, None, None, None, None]
    sdN = np.einsum("eqdk,eqbk->eqbd", f["sig"], dN)    # sigma[d,k] dN_b[k]
    coef = (2.0 * (1.0 - prm.kappa) * f["phi"])[:, :, None, None] * sdN \
        + (2.0 * prm.p * f["phi"])[:, :, None, None] * dN
    Kpu = np.einsum("eqbd,qa->eabd", coef, N) * W[:, None, None, None]
    react = (1.0 - prm.kappa) * f["s"] + 2.0 * prm.p * f["theta"] + prm.Gc / prm.eps
    Kpp = np.einsum("eq,qb,qa->eab", react, N, N) + prm.Gc * prm.eps * np.einsum("eqab->eab", lap)
    Kpp *= W[:, None, None]
    return f["conn"], Kuu, Kpu, Kpp


def jacobian_all(mesh, prm, u, phi, phi_tilde, cells_idx=None):
    """Uncondensed Jacobian on all-node unknowns (u: node*d + c, phi: d*n_nodes + node)."""
    conn, Kuu, Kpu, Kpp = element_matrices(mesh, prm, u, phi, phi_tilde, cells_idx)
    d = mesh.dim
    ne, nv = conn.shape
    n = mesh.n_nodes
    udof = conn[:, :, None] * d + np.arange(d)[None, None, :]      # [e, a, c]
    pdof = d * n + conn                                               # [e, a]
    r1 = np.broadcast_to(udof[:, :, :, None, None], Kuu.shape)
    c1 = np.broadcast_to(udof[:, None, None, :, :], Kuu.shape)
    r2 = np.broadcast_to(pdof[:, :, None, None], Kpu.shape)
    c2 = np.broadcast_to(udof[:, None, :, :], Kpu.shape)
    r3 = np.broadcast_to(pdof[:, :, None], Kpp.shape)
    c3 = np.broadcast_to(pdof[:, None, :], Kpp.shape)
    rows = np.concatenate([r1.ravel(), r2.ravel(), r3.ravel()])
    cols = np.concatenate([c1.ravel(), c2.ravel(), c3.ravel()])
    vals = np.concatenate([Kuu.ravel(), Kpu.ravel(), Kpp.ravel()])
    nt = (d + 1) * n
    return sp.csr_matrix((vals, (rows, cols)), shape=(nt, nt))


def jacobian(mesh, prm, u, phi, phi_tilde):
    """Condensed Jacobian in solve order: J = Cb^T J_all Cb (block lower triangular)."""
    Cb = block_C(mesh)
    J = (Cb.T @ jacobian_all(mesh, prm, u, phi, phi_tilde) @ Cb).tocsr()
    J.sum_duplicates()
    J.sort_indices()
    return J


def expand(mesh, U):
    """Solve-order vector -> (u[n_nodes, d], phi[n_nodes]) on all nodes via C."""
    d = mesh.dim
    nf = mesh.n_free
    uf = U[:d * nf].reshape(nf, d)
    pf = U[d * nf:]
    return mesh.C @ uf, mesh.C @ pf


def restrict(mesh, u, phi):
    """All-node state -> solve-order vector (values at the free nodes)."""
    return np.concatenate([u[mesh.free].ravel(), phi[mesh.free]])

"""Active set, elimination, exact linear solve and the Newton / active-set loop (Section 3).

Active set (commented algorithm of Section 3, step 2; the printed rule is garbled).
Reading from the KKT conditions of phi <= phi_old: the multiplier density is
lambda_i = -R_phi,i / B_ii with B the lumped (row-summed, condensed) phi mass, and
    i in A  <=>  lambda_i + c (phi_i - phi_old_i) > tau,
with c = 1 and tau = 1e-10 G_c / eps, so that far-field DoFs whose lambda is 0 up to
rounding are deterministically inactive.

Elimination (step 4): Dirichlet u DoFs (target u = 0) and active phi DoFs (target
phi_old) are fixed; with delta*_i = target_i - current_i the masked system keeps the
original diagonal d_i, zeroes the rest of row and column i, sets F_i = d_i delta*_i and
moves the column into the right-hand side of the other rows.

Exact linear solve: the Jacobian is block lower triangular (M_u_phi = 0), so
    M_uu du = F_u,   M_phiphi dphi = F_phi - M_phiu du,
each solved by sparse LU (scipy SuperLU as a library step), or the whole masked J by
dense LU for tiny meshes.  This is a different solver from the GPU's FGMRES + AMG.

Newton loop (steps 1-6 with the stop rule "active set unchanged and residual < TOL"):
line search omega in {1, 1/2, ..., 2^-8} on the DoFs that are not fixed, first omega with
||R~(U + omega dU)||_2 < ||R~(U)||_2 (else 2^-8); the fixed DoFs take their constraint values
at every trial (0 for Dirichlet u, phi_old for active phi: the elimination of step 4 fixes
them, and a damped step would leave an active DoF off phi_old while R~, which omits its row,
reports convergence); stop when A_k = A_{k-1} and
||R~(U^k)||_2 <= max(tol ||R~(U^0)||_2, atol), at most max_it iterations.  The paper's
rule compares R~ with an absolute TOL (atol); the relative part serves a step that starts
far from equilibrium, the absolute part a step that starts at it (a later loading step at
an unchanged load), whose R~(U^0) is already at rounding level.  R~ is R with fixed rows
zeroed.  Cycle rule (the paper only says alternating indices are detected and
constrained): a phi DoF whose membership flips twice within three consecutive iterates
is frozen active for the rest of the loading step.  Status at the iteration cap: "cycle"
when the residual part of the stop test is met and only the active set still changes,
else "noconv".

Pinned by tests/test_oracle_newton.py: dense LU of the full masked J against the block
forward substitution; KKT conditions at the Newton fixed point; brute-force enumeration of
all active sets of the linearised problem on a tiny mesh; the cycle rule on every
membership sequence of three iterates (only in-out-in and out-in-out freeze, frozen DoFs
stay active), and on a seeded problem whose iterates alternate: without the rule the loop
cycles to the cap with a converged residual, with it the two alternating DoFs are frozen and
the loop stops.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def active_set(mesh, prm, R, B, phi, phi_old):
    """Boolean mask over the free phi DoFs and the margin lambda + c(phi-phi_old) - tau."""
    d = mesh.dim
    nf = mesh.n_free
    Rp = R[d * nf:]
    lam = -Rp / B
    pf = phi[mesh.free]
    pof = phi_old[mesh.free]
    margin = lam + prm.c_pdas * (pf - pof) - prm.tau
    return margin > 0.0, margin


def fixed_dofs(mesh, active, u, phi, phi_old):
    """Mask of fixed solve-order DoFs and their target increments delta*."""
    d = mesh.dim
    nf = mesh.n_free
    fixed = np.zeros((d + 1) * nf, dtype=bool)
    target = np.zeros((d + 1) * nf)
    dir_f = mesh.dirichlet[mesh.free]
    ufix = np.repeat(dir_f, d)
    fixed[:d * nf] = ufix
    target[:d * nf] = np.where(ufix, -u[mesh.free].ravel(), 0.0)
    fixed[d * nf:] = active
    target[d * nf:] = np.where(active, phi_old[mesh.free] - phi[mesh.free], 0.0)
    return fixed, target


def fixed_values(mesh, active, phi_old):
    """Values the fixed solve-order DoFs take after an update: 0 for Dirichlet u DoFs and
    phi_old for active phi DoFs (the elimination of step 4 fixes them there)."""
    d = mesh.dim
    nf = mesh.n_free
    val = np.zeros((d + 1) * nf)
    val[d * nf:] = np.where(active, phi_old[mesh.free], 0.0)
    return val


def mask_system(J, R, fixed, target):
    """Eliminate fixed rows/columns (step 4): returns (J_masked CSR, F)."""
    J = J.tocsr()
    diag = J.diagonal()
    keep = (~fixed).astype(np.float64)
    F = -R.copy()
    F -= J @ np.where(fixed, target, 0.0)
    Dk = sp.diags(keep)
    Jm = (Dk @ J @ Dk + sp.diags(np.where(fixed, diag, 0.0))).tocsr()
    F = np.where(fixed, diag * target, F)
    Jm.eliminate_zeros()
    Jm.sort_indices()
    return Jm, F


def alternating(a_before, a_prev, a_new):
    """DoFs whose membership flips twice over three consecutive iterates: in, out, in or
    out, in, out (the alternating active-set indices Section 3 detects)."""
    return (a_before != a_prev) & (a_prev != a_new)


def freeze(a_before, a_prev, a_new, frozen):
    """Cycle rule of Section 3 (alternating indices are constrained): every alternating DoF
    joins `frozen` for the rest of the loading step, and frozen DoFs are active.  Returns the
    new (active, frozen) pair; the inputs are not modified."""
    frozen = frozen | alternating(a_before, a_prev, a_new)
    return a_new | frozen, frozen


def masked_residual_norm(R, fixed):
    return float(np.linalg.norm(np.where(fixed, 0.0, R)))


def solve_block(mesh, Jm, F):
    """Exact solve by block forward substitution (M_u_phi = 0)."""
    d = mesh.dim
    nu = d * mesh.n_free
    Juu = Jm[:nu, :nu].tocsc()
    Jpu = Jm[nu:, :nu]
    Jpp = Jm[nu:, nu:].tocsc()
    du = spla.splu(Juu).solve(F[:nu])
    dp = spla.splu(Jpp).solve(F[nu:] - Jpu @ du)
    return np.concatenate([du, dp])


def solve_dense(Jm, F):
    """Dense LU of the full masked Jacobian (tiny meshes only)."""
    return np.linalg.solve(Jm.toarray(), F)


class StepResult:
    pass


def newton_step_system(mesh, prm, u, phi, phi_old, phi_tilde):
    """Steps 1-4 at one state: R, active set, masked (J, F) and the fixed mask."""
    R, B = fem.residual(mesh, prm, u, phi, phi_tilde)
    active, margin = active_set(mesh, prm, R, B, phi, phi_old)
    J = fem.jacobian(mesh, prm, u, phi, phi_tilde)
    fixed, target = fixed_dofs(mesh, active, u, phi, phi_old)
    Jm, F = mask_system(J, R, fixed, target)
    out = StepResult()
    out.R, out.B, out.active, out.margin, out.J = R, B, active, margin, J
    out.fixed, out.target, out.Jm, out.F = fixed, target, Jm, F
    return out


def newton_loop(mesh, prm, u0, phi0, phi_old, phi_tilde, tol=1e-8, max_it=30,
                linear_solve=None, ls_max=8, atol=0.0, freeze_cycles=True):
    """Full Newton / active-set loop for one loading step (Section 3 algorithm).
    freeze_cycles=False leaves the cycle rule out (the library's diagnostic option)."""
    if linear_solve is None:
        linear_solve = lambda Jm, F: solve_block(mesh, Jm, F)
    d = mesh.dim
    nf = mesh.n_free
    U = fem.restrict(mesh, u0, phi0)
    u, phi = fem.expand(mesh, U)
    frozen = np.zeros(nf, dtype=bool)
    history = []
    R, B = fem.residual(mesh, prm, u, phi, phi_tilde)
    active, _ = active_set(mesh, prm, R, B, phi, phi_old)
    active |= frozen
    fixed, target = fixed_dofs(mesh, active, u, phi, phi_old)
    r0 = masked_residual_norm(R, fixed)
    log = []
    prev_active = None
    it = 0
    converged = False
    while it < max_it:
        history.append(active.copy())
        J = fem.jacobian(mesh, prm, u, phi, phi_tilde)
        Jm, F = mask_system(J, R, fixed, target)
        dU = linear_solve(Jm, F)
        rk = masked_residual_norm(R, fixed)
        omega = 2.0 ** -ls_max
        fval = fixed_values(mesh, active, phi_old)
        for m in range(ls_max + 1):
            w = 2.0 ** -m
            Ut = np.where(fixed, fval, U + w * dU)
            ut, pt = fem.expand(mesh, Ut)
            Rt, _ = fem.residual(mesh, prm, ut, pt, phi_tilde)
            if masked_residual_norm(Rt, fixed) < rk:
                omega = w
                break
        U = np.where(fixed, fval, U + omega * dU)
        u, phi = fem.expand(mesh, U)
        it += 1
        R, B = fem.residual(mesh, prm, u, phi, phi_tilde)
        new_active, _ = active_set(mesh, prm, R, B, phi, phi_old)
        if freeze_cycles and len(history) >= 2:
            new_active, frozen = freeze(history[-2], history[-1], new_active, frozen)
        else:
            new_active = new_active | frozen
        fixed, target = fixed_dofs(mesh, new_active, u, phi, phi_old)
        rn = masked_residual_norm(R, fixed)
        log.append(dict(it=it, omega=omega, res=rn, n_active=int(new_active.sum()),
                        changed=int((new_active != active).sum())))
        same = np.array_equal(new_active, active)
        active = new_active
        res_ok = rn <= max(tol * r0, atol)
        if same and res_ok:
            converged = True
            break
    # the iteration cap: a loop held back only by a still-changing active set is a cycle the
    # freeze did not resolve, anything else is plain non-convergence
    status = "ok" if converged else ("cycle" if res_ok else "noconv")
    return dict(u=u, phi=phi, U=U, active=active, iterations=it, converged=converged,
                r0=r0, res=rn if it else r0, log=log, frozen=frozen, status=status)

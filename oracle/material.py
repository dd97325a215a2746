"""Material data of Formulation 1 (Section 2) and the parameters of Section 4.

The paper only names "Lame coefficients" mu_s, lambda_s and gives E=1, nu=0.2 (Section 4).
Reading: the standard isotropic relations; in 2d the problem is plane strain, which is
the setting in which Sneddon's forms carry the factor (1 - nu^2)/E (Section 4).

Pinned by tests/test_oracle_basics.py (test_lame_relations: nu recovered from
lambda/(2(lambda+mu)) and E from mu(3 lambda + 2 mu)/(lambda + mu); test_appendix_constants).
"""
from dataclasses import dataclass


def lame(E, nu):
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


@dataclass
class Params:
    """Per-instance constants: E, nu, G_c, kappa, eps, p and the active-set constants.

    c_pdas and tau_pdas define the active-set test
    lambda_i + c_pdas (phi_i - phi_old_i) > tau_pdas  (Section 3, commented algorithm,
    step 2; reading of the garbled rule).  tau_pdas = 0 means 1e-10 * G_c / eps.
    """
    E: float = 1.0
    nu: float = 0.2
    Gc: float = 1.0
    kappa: float = 1e-10
    eps: float = 1.0 / 16.0
    p: float = 1e-3
    c_pdas: float = 1.0
    tau_pdas: float = 0.0

    @property
    def mu(self):
        return lame(self.E, self.nu)[0]

    @property
    def lam(self):
        return lame(self.E, self.nu)[1]

    @property
    def tau(self):
        return self.tau_pdas if self.tau_pdas > 0.0 else 1e-10 * self.Gc / self.eps

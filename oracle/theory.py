"""Closed-form bounds of Sec. 3.4 (convergence analysis).

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

* Corollary "Computable Fourier spectral enclosure": beta_N = alpha +
  theta k C_hat max|xi|^2, q_bar(lambda) = max(|lambda-alpha|/(lambda+alpha),
  |lambda-beta|/(lambda+beta)), minimized at lambda_bd = sqrt(alpha beta_N).
* Theorem "Full saddle two-step contraction": gamma_m, vartheta_2,
  kappa_lambda.
* Corollary "Uniform iteration bound": 2 ceil(log(kappa/eps)/log(1/vartheta)).
* Remark "Bounded exchange stiffness versus an explicit CFL condition":
  forward Euler on the linearized exchange flow needs k C_hat max|xi|^2 <= 2 alpha.
"""

import math


def beta_n(alpha, theta, dt, c_hat, max_symbol):
    return alpha + theta * dt * c_hat * max_symbol


def q_bar(lam, alpha, beta):
    return max(abs(lam - alpha) / (lam + alpha), abs(lam - beta) / (lam + beta))


def lambda_bd(alpha, beta):
    return math.sqrt(alpha * beta)


def gamma_m(lam, m_min, m_max=None):
    """min over nodal norms in [m_min, m_max] of 2 lam s / (lam^2 + s^2)."""
    f = lambda s: 2.0 * lam * s / (lam * lam + s * s)
    return f(m_min) if m_max is None else min(f(m_min), f(m_max))


def vartheta2(q_h, gamma):
    return math.sqrt(1.0 - (1.0 - q_h * q_h) * gamma * gamma / (gamma * gamma + 1.0 + q_h * q_h))


def kappa(lam, m_min, m_max):
    return math.sqrt((lam * lam + m_max * m_max) / (lam * lam + m_min * m_min))


def iteration_bound(kap, theta2, eps):
    return 2 * math.ceil(math.log(kap / eps) / math.log(1.0 / theta2))


def explicit_limit_ratio(dt, c_hat, max_symbol, alpha):
    """k C_hat max|xi|^2 / (2 alpha): how many times the explicit limit."""
    return dt * c_hat * max_symbol / (2.0 * alpha)


def dt_for_ratio(ratio, alpha, c_hat, max_symbol):
    """Time step that is ``ratio`` times the explicit exchange limit."""
    return ratio * 2.0 * alpha / (c_hat * max_symbol)

"""Planted mistakes in the oracle must fail at least one pin.

Each case monkeypatches one plausible error into the oracle (transposed
operand, dropped term, wrong sign, wrong index) and re-runs a pin from
test_oracle_pins; the pin must now fail.  Runs on the CPU only.
"""
import math

import numpy as np
import pytest

from oracle import fcgle_oracle as O
import tests.test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_transposed_eigenvectors_are_caught(monkeypatch):
    orig = O.apply_f

    def bad(kind, theta, V, Qs, lams, params):
        Vhat = O.tucker(V, Qs)  # Q instead of Q^T
        return O.tucker(O.f_grid(kind, theta, lams, params) * Vhat, [Q.T for Q in Qs])

    monkeypatch.setattr(O, "apply_f", bad)
    assert _fails(pins.test_apply_f_matches_brute_force, (7, 9), "exp")
    monkeypatch.setattr(O, "apply_f", orig)


def test_dropped_gamma_term_is_caught(monkeypatch):
    def bad(t, U, params, source=None):
        _, _, gamma, kappa, zeta = params
        out = -(kappa + 1j * zeta) * (np.abs(U) ** 2) * U
        if source is not None:
            out = out + source(t, U.shape)
        return out

    monkeypatch.setattr(O, "g_nonlin", bad)
    assert _fails(pins.test_manufactured_solution_solves_the_semidiscrete_ode)


def test_wrong_sign_of_D_is_caught(monkeypatch):
    def bad(alpha, n, h, fd_order=2):
        g = O.fd2_weights(alpha, n)
        import scipy.linalg as sla
        return (h ** -alpha) * sla.toeplitz(g)

    monkeypatch.setattr(O, "diff_matrix", bad)
    assert _fails(pins.test_D_symmetric_toeplitz_negative_definite, 1.5)


def test_recurrence_index_slip_is_caught(monkeypatch):
    def bad(alpha, n):
        g = np.empty(n)
        g[0] = math.gamma(alpha + 1) / math.gamma(alpha / 2 + 1) ** 2
        for k in range(1, n):
            g[k] = (1.0 - (alpha + 1) / (alpha / 2 + k + 1)) * g[k - 1]
        return g

    monkeypatch.setattr(O, "fd2_weights", bad)
    assert _fails(pins.test_fd2_recurrence_matches_gamma_definition, 1.5)


def test_phi_series_off_by_one_is_caught(monkeypatch):
    def bad(l, z):
        z = np.asarray(z, dtype=np.complex128)
        if l == 0:
            return np.exp(z)
        acc = np.zeros_like(z)
        for k in range(39, -1, -1):
            acc = acc * z + 1.0 / math.factorial(k + l - 1)
        return acc

    monkeypatch.setattr(O, "phi", bad)
    assert _fails(pins.test_phi_matches_high_precision_definition, 1)


def test_lbdf2_wrong_extrapolation_is_caught(monkeypatch):
    def bad(P, U, Uprev, t, tau):
        rhs = (4.0 / 3.0) * U - (1.0 / 3.0) * Uprev + (2.0 * tau / 3.0) * P.g(t + tau, U)
        return P.f("inv", 2.0 * tau / 3.0, rhs)

    monkeypatch.setattr(O, "step_lbdf2", bad)
    assert _fails(pins.test_observed_temporal_order_on_manufactured_solution, "lbdf2", 2)


def test_adjoint_missing_conjugate_is_caught(monkeypatch):
    orig = O.expeuler_vjp

    def bad(P, U, Ubar_next, t, tau):
        ubar, pbar = orig(P, U, Ubar_next, t, tau)
        nu, eta, gamma, kappa, zeta = P.params
        c = kappa + 1j * zeta
        z = tau * (nu + 1j * eta) * O.ell_grid(P.lams)
        a_hat = O.tucker(Ubar_next, [Q.T for Q in P.Qs])
        w = tau * O.tucker(np.conj(O.phi(1, z)) * a_hat, P.Qs)
        # replace -c u^2 conj(w) by -c u^2 w
        ubar = ubar + c * U * U * np.conj(w) - c * U * U * w
        return ubar, pbar

    monkeypatch.setattr(O, "expeuler_vjp", bad)
    assert _fails(pins.test_exp_euler_adjoint_matches_central_differences)


def test_flow_phi1_argument_slip_is_caught(monkeypatch):
    # phi_1(gamma t) instead of phi_1(2 gamma t) in the exact nonlinear flow
    def bad(W, t, params):
        _, _, gamma, kappa, zeta = params
        tp1 = t * O.phi(1, np.array([gamma * t])).real[0]
        m = np.abs(W) ** 2
        return np.exp(t * gamma - (kappa + 1j * zeta) / (2.0 * kappa) * np.log(1.0 + 2.0 * tp1 * kappa * m)) * W

    monkeypatch.setattr(O, "nonlinear_flow", bad)
    assert _fails(pins.test_nonlinear_flow_solves_its_ode, (0.0, 0.0, 1.0, 1.0, 2.0))


def test_flow_phase_sign_is_caught(monkeypatch):
    orig = O.nonlinear_flow

    def bad(W, t, params):
        nu, eta, gamma, kappa, zeta = params
        return orig(W, t, (nu, eta, gamma, kappa, -zeta))

    monkeypatch.setattr(O, "nonlinear_flow", bad)
    assert _fails(pins.test_nonlinear_flow_solves_its_ode, (0.0, 0.0, 1.3, 0.0, 0.9))


def test_strang_full_step_flows_are_caught(monkeypatch):
    # both nonlinear substeps taken with tau instead of tau / 2
    def bad(P, U, t, tau):
        return O.nonlinear_flow(P.f("exp", tau, O.nonlinear_flow(U, tau, P.params)), tau, P.params)

    monkeypatch.setattr(O, "step_strang", bad)
    assert _fails(pins.test_strang_is_second_order_against_the_ode_solution)


def test_riesz_normalisation_slip_is_caught(monkeypatch):
    # cos(alpha pi) instead of cos(alpha pi / 2) in the Riesz normalisation
    def bad(x, alpha):
        x = np.asarray(x, dtype=np.float64)
        return -(O.rl_left_bump(x, alpha) + O.rl_left_bump(-x, alpha)) / (2.0 * math.cos(alpha * math.pi))

    monkeypatch.setattr(O, "riesz_bump", bad)
    assert _fails(pins.test_fd2_matrix_converges_to_the_riesz_derivative_of_the_bump)


def test_rl_gamma_ratio_slip_is_caught(monkeypatch):
    # Gamma(p) / Gamma(p - alpha) instead of Gamma(p + 1) / Gamma(p + 1 - alpha)
    from scipy.special import gamma as Gam

    def bad(x, alpha):
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros_like(x)
        for k in range(5):
            p = 4 + k
            c = math.comb(4, k) * 2.0 ** (4 - k) * (-1.0) ** k
            out = out + c * Gam(p) / Gam(p - alpha) * (1.0 + x) ** (p - alpha)
        return out

    monkeypatch.setattr(O, "rl_left_bump", bad)
    assert _fails(pins.test_rl_derivative_of_the_bump_matches_its_integral_definition, 1.5)


def test_krogstad_phi3_weight_slip_is_caught(monkeypatch):
    # -4 d_4 instead of +4 d_4 in the phi_3 term of the last stage
    def bad(P, U, t, tau):
        g_n = P.g(t, U)
        f_n = O.apply_K(U, P.Ds, P.params) + g_n
        half = U + 0.5 * tau * P.f("phi1", 0.5 * tau, f_n)
        d2 = P.g(t + 0.5 * tau, half) - g_n
        u3 = half + tau * P.f("phi2", 0.5 * tau, d2)
        d3 = P.g(t + 0.5 * tau, u3) - g_n
        full = U + tau * P.f("phi1", tau, f_n)
        d4 = P.g(t + tau, full + 2.0 * tau * P.f("phi2", tau, d3)) - g_n
        return (full + tau * P.f("phi2", tau, 2.0 * d2 + 2.0 * d3 - d4)
                + tau * P.f("phi3", tau, -4.0 * d2 - 4.0 * d3 - 4.0 * d4))

    monkeypatch.setattr(O, "step_krogstad", bad)
    assert _fails(pins.test_krogstad_is_fourth_order_on_the_manufactured_solution)

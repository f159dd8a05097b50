"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the Gamma
definition of the FD weights, alpha -> 2 closed forms (classical 3- and 5-point
stencils, Dirichlet-Laplacian eigenpairs), a high-precision evaluation of the
phi-functions from their definition, brute force on the assembled Kronecker
sum (expm / solve / augmented expm), the Kronecker-product exponential, the
2-D Sylvester form of the inverse, invariants, observed temporal orders on a
manufactured solution, and central finite differences for the adjoint.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fcgle_oracle as O
from workloads import grid_axes, random_complex, sech_product

PARAMS = (1.0, 0.5, 1.0, 1.0, 0.5)


# --- Section 2: FD weights and D ------------------------------------------------------

@pytest.mark.parametrize("alpha", [1.1, 1.3, 1.5, 1.7, 1.9, 1.99])
def test_fd2_recurrence_matches_gamma_definition(alpha):
    n = 30
    g_rec = O.fd2_weights(alpha, n)
    g_def = O.fd2_weights_gamma(alpha, n)
    assert np.max(np.abs(g_rec - g_def)) <= 1e-13 * np.max(np.abs(g_def))


def test_fd2_alpha2_is_three_point_laplacian():
    g = O.fd2_weights(2.0, 12)
    np.testing.assert_allclose(g, [2.0, -1.0] + [0.0] * 10, atol=1e-15)


def test_fd4_alpha2_is_five_point_stencil():
    g = O.fd4_weights(2.0, 12)
    np.testing.assert_allclose(g, [2.5, -4.0 / 3.0, 1.0 / 12.0] + [0.0] * 9, atol=1e-15)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_D_symmetric_toeplitz_negative_definite(alpha):
    n, h = 40, 0.3
    D = O.diff_matrix(alpha, n, h)
    assert np.array_equal(D, D.T)
    for k in range(1, n):
        assert np.all(np.diag(D, k) == D[0, k])
    assert np.all(np.linalg.eigvalsh(D) < 0)
    # the weight sum is positive and g_k < 0 for k >= 1 (diagonal dominance)
    g = O.fd2_weights(alpha, n)
    assert g[0] > 0 and np.all(g[1:] < 0) and g[0] + 2 * np.sum(g[1:]) > 0


def test_eig_alpha2_dirichlet_laplacian_closed_form():
    n, h = 17, 0.2
    lam, Q = O.eig(O.diff_matrix(2.0, n, h))
    k = np.arange(1, n + 1)
    lam_exact = -(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n + 1))) ** 2
    np.testing.assert_allclose(np.sort(lam), np.sort(lam_exact), rtol=1e-13)
    j = np.arange(1, n + 1)[:, None]
    Qex = np.sqrt(2.0 / (n + 1)) * np.sin(j * k[None, :] * np.pi / (n + 1))
    # match columns (eigenvalues distinct); sign is arbitrary
    order = np.argsort(lam)
    order_ex = np.argsort(lam_exact)
    for a, b in zip(order, order_ex):
        s = np.sign(Q[:, a] @ Qex[:, b])
        np.testing.assert_allclose(s * Q[:, a], Qex[:, b], atol=1e-12)


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_eig_reconstruction_and_orthogonality(alpha):
    n, h = 64, 0.1
    D = O.diff_matrix(alpha, n, h)
    lam, Q = O.eig(D)
    assert np.linalg.norm(Q @ np.diag(lam) @ Q.T - D) <= 1e-14 * n * np.linalg.norm(D)
    # orthogonal to the rounding of its FP64 entries (spectral norm), see oracle.eig
    assert np.linalg.norm(Q.T @ Q - np.eye(n), 2) <= 1.5e-15
    assert np.all(lam < 0)


# --- phi-functions ----------------------------------------------------------------------

def _phi_mp(l, z):
    """phi_l from its definition in 60-digit arithmetic (recurrence is exact enough there)."""
    with mpmath.workdps(60):
        zz = mpmath.mpc(z.real, z.imag)
        if zz == 0:
            return complex(1 / mpmath.factorial(l))
        p = mpmath.exp(zz)
        for j in range(1, l + 1):
            p = (p - 1 / mpmath.factorial(j - 1)) / zz
        return complex(p)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_phi_matches_high_precision_definition(l):
    rng = np.random.default_rng(3)
    mags = np.concatenate([10.0 ** rng.uniform(-9, 1.2, 200), [0.999, 1.0, 1.001]])
    args = rng.uniform(0, 2 * np.pi, mags.size)
    z = mags * np.exp(1j * args)
    got = O.phi(l, z)
    ref = np.array([_phi_mp(l, zz) for zz in z])
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 2e-14


def test_phi_at_zero():
    for l in range(4):
        assert O.phi(l, np.array([0.0]))[0] == pytest.approx(1.0 / math.factorial(l), rel=0, abs=0)


# --- Section 3: matrix function actions ---------------------------------------------------

def _problem(n, seed, params=PARAMS):
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(1.1, 1.95, len(n))
    h = rng.uniform(0.05, 0.5, len(n))
    Ds, Qs, lams = O.setup(n, alpha, h)
    return Ds, Qs, lams


def test_kron_order_matches_mode_products():
    Ds, Qs, lams = _problem((4, 5, 3), 0)
    V = random_complex((4, 5, 3), 1)
    K = O.kron_sum(Ds, PARAMS)
    np.testing.assert_allclose((K @ V.ravel()).reshape(V.shape), O.apply_K(V, Ds, PARAMS), rtol=0, atol=1e-9)


@pytest.mark.parametrize("n", [(7, 9), (5, 6, 4), (3, 4, 2, 3)])
@pytest.mark.parametrize("kind", ["inv", "exp", "phi1", "phi2", "phi3"])
def test_apply_f_matches_brute_force(n, kind):
    Ds, Qs, lams = _problem(n, 10 + len(n))
    V = random_complex(n, 2)
    theta = 3e-3
    got = O.apply_f(kind, theta, V, Qs, lams, PARAMS)
    ref = O.brute_apply(kind, theta, V, Ds, PARAMS)
    assert O.rel_l2(got, ref) <= 1e-12


def test_apply_exp_matches_kronecker_product_of_1d_exponentials():
    n = (16, 20, 12)
    Ds, Qs, lams = _problem(n, 5)
    V = random_complex(n, 6)
    got = O.apply_f("exp", 1e-2, V, Qs, lams, PARAMS)
    ref = O.exp_neudecker(1e-2, V, Ds, PARAMS)
    assert O.rel_l2(got, ref) <= 1e-12


def test_apply_inv_matches_sylvester_2d():
    n = (24, 31)
    Ds, Qs, lams = _problem(n, 7)
    V = random_complex(n, 8)
    theta = 2e-2
    c = PARAMS[0] + 1j * PARAMS[1]
    a = 0.5 * np.eye(n[0]) - theta * c * Ds[0]
    b = (0.5 * np.eye(n[1]) - theta * c * Ds[1]).T
    ref = sla.solve_sylvester(a, b, V)
    got = O.apply_f("inv", theta, V, Qs, lams, PARAMS)
    assert O.rel_l2(got, ref) <= 1e-11


def test_phi1_identity_with_dense_operator():
    n = (20, 14, 9)
    Ds, Qs, lams = _problem(n, 9)
    V = random_complex(n, 10)
    theta = 5e-3
    lhs = theta * O.apply_K(O.apply_f("phi1", theta, V, Qs, lams, PARAMS), Ds, PARAMS)
    rhs = O.apply_f("exp", theta, V, Qs, lams, PARAMS) - V
    assert O.rel_l2(lhs, rhs) <= 1e-11


def test_exp_is_unitary_when_dispersive():
    params = (0.0, 1.3, 0.0, 0.0, 0.7)
    n = (12, 10, 8)
    Ds, Qs, lams = _problem(n, 11, params)
    V = random_complex(n, 12)
    out = O.apply_f("exp", 0.3, V, Qs, lams, params)
    assert abs(np.linalg.norm(out) / np.linalg.norm(V) - 1.0) <= 1e-13


# --- schemes -------------------------------------------------------------------------------

def _manufactured(n, domain, alpha, params=PARAMS):
    axes = grid_axes(n, domain)
    h = [(b - a) / (m + 1) for (a, b), m in zip(domain, n)]
    U0 = sech_product(axes, [1.0] + [0.0] * (len(n) - 1))
    P = O.Problem(n, alpha, h, params)
    P.source = O.manufactured_source(U0, P.Ds, params)
    return P, U0


def test_manufactured_solution_solves_the_semidiscrete_ode():
    P, U0 = _manufactured((9, 8, 7), ((-8.0, 8.0),) * 3, (1.3, 1.6, 1.8))
    for t in (0.0, 0.37):
        u = math.exp(-t) * U0
        dudt = -math.exp(-t) * U0
        rhs = O.apply_K(u, P.Ds, P.params) + P.g(t, u)
        assert np.linalg.norm(dudt - rhs) <= 1e-12 * np.linalg.norm(dudt)


@pytest.mark.parametrize("scheme,order", [("exp_euler", 1), ("lawson", 1), ("lie", 1), ("lbdf2", 2)])
def test_observed_temporal_order_on_manufactured_solution(scheme, order):
    P, U0 = _manufactured((10, 12, 8), ((-8.0, 8.0),) * 3, (1.3, 1.6, 1.8))
    T = 0.5
    errs = []
    taus = [2e-2, 1e-2, 5e-3, 2.5e-3]
    for tau in taus:
        steps = int(round(T / tau))
        U = O.run(P, scheme, U0, tau, steps)
        errs.append(O.rel_l2(U, math.exp(-T) * U0))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(taus))
    assert abs(slopes[-1] - order) <= 0.1, (errs, slopes)


def test_first_order_norm_drift_vanishes_with_tau():
    # nu = gamma = kappa = 0, s = 0: the flow conserves the L2 norm; exponential Euler is
    # exact on the linear part, so the drift comes from the nonlinear term only and is O(tau).
    params = (0.0, 1.0, 0.0, 0.0, 1.0)
    n = (16, 12)
    axes = grid_axes(n, ((-10.0, 10.0),) * 2)
    U0 = sech_product(axes, (1.0, 1.0))
    P = O.Problem(n, (1.5, 1.5), [20.0 / 17, 20.0 / 13], params)
    drifts = []
    for tau in (4e-2, 2e-2, 1e-2):
        U = O.run(P, "exp_euler", U0, tau, int(round(0.4 / tau)))
        drifts.append(abs(np.linalg.norm(U) / np.linalg.norm(U0) - 1.0))
    slopes = np.diff(np.log(drifts)) / np.log(0.5)
    assert np.all(np.abs(slopes - 1.0) < 0.15), (drifts, slopes)


# --- adjoint -------------------------------------------------------------------------------

def _loss(params, U0, n, alpha, h, target, tau, steps):
    P = O.Problem(n, alpha, h, params)
    U = O.run(P, "exp_euler", U0, tau, steps)
    return float(np.sum(np.abs(U - target) ** 2))


def test_exp_euler_adjoint_matches_central_differences():
    n = (8, 7, 6)
    alpha = (1.5, 1.4, 1.6)
    h = (20.0 / 9, 20.0 / 8, 20.0 / 7)
    axes = grid_axes(n, ((-10.0, 10.0),) * 3)
    U0 = sech_product(axes, (1.0, 0.0, 0.0))
    tau, steps = 1e-2, 6
    pert = np.array(PARAMS) + np.array([0.1, -0.1, 0.1, -0.1, 0.1])
    target = O.run(O.Problem(n, alpha, h, tuple(pert)), "exp_euler", U0, tau, steps)
    P = O.Problem(n, alpha, h, PARAMS)
    L, ubar0, pbar = O.expeuler_loss_and_grad(P, U0, target, tau, steps)
    fd_h = 1e-4
    # parameters
    for i in range(5):
        pp = np.array(PARAMS); pp[i] += fd_h
        pm = np.array(PARAMS); pm[i] -= fd_h
        fd = (_loss(tuple(pp), U0, n, alpha, h, target, tau, steps)
              - _loss(tuple(pm), U0, n, alpha, h, target, tau, steps)) / (2 * fd_h)
        assert abs(fd - pbar[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, pbar[i])
    # initial state, along random complex unit directions
    rng = np.random.default_rng(5)
    for _ in range(4):
        dlt = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        dlt /= np.linalg.norm(dlt)
        fd = (_loss(PARAMS, U0 + fd_h * dlt, n, alpha, h, target, tau, steps)
              - _loss(PARAMS, U0 - fd_h * dlt, n, alpha, h, target, tau, steps)) / (2 * fd_h)
        an = float(np.real(np.vdot(ubar0, dlt)))
        assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (fd, an)


# --- Strang splitting (Section 4, eq. Strang) ----------------------------------------------

def _ode_solution(rhs, y0, T):
    """Adaptive 8th-order Runge-Kutta (scipy DOP853) on the real view of a complex system."""
    from scipy.integrate import solve_ivp
    y0 = np.asarray(y0, np.complex128)
    shape = y0.shape

    def f(_, y):
        w = (y[: y.size // 2] + 1j * y[y.size // 2:]).reshape(shape)
        d = rhs(w).ravel()
        return np.concatenate([d.real, d.imag])

    sol = solve_ivp(f, (0.0, T), np.concatenate([y0.real.ravel(), y0.imag.ravel()]), method="DOP853",
                    rtol=1e-13, atol=1e-15)
    assert sol.success
    y = sol.y[:, -1]
    return (y[: y.size // 2] + 1j * y[y.size // 2:]).reshape(shape)


@pytest.mark.parametrize("params", [(0.0, 0.0, 1.0, 1.0, 2.0), (0.0, 0.0, -0.7, 0.4, -1.3),
                                    (0.0, 0.0, 0.0, 0.8, 0.5), (0.0, 0.0, 1.3, 0.0, 0.9),
                                    (0.0, 0.0, 0.0, 0.0, 1.0)])
def test_nonlinear_flow_solves_its_ode(params):
    _, _, gamma, kappa, zeta = params
    W0 = 1.5 * random_complex((40,), 3)
    for t in (0.05, 0.7):
        ref = _ode_solution(lambda w: gamma * w - (kappa + 1j * zeta) * np.abs(w) ** 2 * w, W0, t)
        assert O.rel_l2(O.nonlinear_flow(W0, t, params), ref) <= 1e-11


def test_nonlinear_flow_is_a_semigroup():
    params = (0.3, 0.2, 0.9, 0.6, -1.1)
    W0 = 2.0 * random_complex((5, 6), 4)
    a = O.nonlinear_flow(O.nonlinear_flow(W0, 0.13, params), 0.29, params)
    assert O.rel_l2(a, O.nonlinear_flow(W0, 0.42, params)) <= 1e-14


def test_strang_conserves_the_norm_when_dispersive():
    # nu = gamma = kappa = 0, s = 0: e^{tau K} is unitary (i eta D anti-Hermitian) and the flow is
    # a pointwise phase, so every Strang step keeps the L2 norm up to rounding
    params = (0.0, 1.0, 0.0, 0.0, 1.0)
    n = (16, 12)
    axes = grid_axes(n, ((-10.0, 10.0),) * 2)
    U0 = sech_product(axes, (1.0, 1.0))
    P = O.Problem(n, (1.2, 1.8), [20.0 / 17, 20.0 / 13], params)
    U = O.run(P, "strang", U0, 0.05, 40)
    assert abs(np.linalg.norm(U) / np.linalg.norm(U0) - 1.0) <= 1e-13


def test_strang_is_second_order_against_the_ode_solution():
    # the paper's second example (no source) on a small grid; reference: the semi-discrete ODE
    # u' = K u + g(u) integrated by an adaptive solver with K assembled densely
    params = (1.0, 1.0, 1.0, 1.0, 1.0)
    n = (10, 12)
    dom = ((-10.0, 10.0),) * 2
    h = [(b - a) / (m + 1) for (a, b), m in zip(dom, n)]
    U0 = sech_product(grid_axes(n, dom), (1.0, 1.0))
    P = O.Problem(n, (1.2, 1.8), h, params)
    K = O.kron_sum(P.Ds, params)
    T = 0.5
    ref = _ode_solution(lambda w: (K @ w.ravel()).reshape(n) + O.g_nonlin(0.0, w, params), U0, T)
    taus = [0.1, 0.05, 0.025, 0.0125]
    errs = [O.rel_l2(O.run(P, "strang", U0, tau, int(round(T / tau))), ref) for tau in taus]
    slopes = np.diff(np.log(errs)) / np.diff(np.log(taus))
    assert abs(slopes[-1] - 2.0) <= 0.1, (errs, slopes)


def test_strang_rejects_a_source():
    P, U0 = _manufactured((6, 5), ((-8.0, 8.0),) * 2, (1.3, 1.6))
    with pytest.raises(ValueError):
        O.step_strang(P, U0, 0.0, 0.01)


# --- the paper's Example 1: continuous source and printed errors ---------------------------

def _bump_second_derivative(x):
    # f = (1 - x^2)^4: f' = -8x (1 - x^2)^3, f'' = -8 (1 - x^2)^3 + 48 x^2 (1 - x^2)^2
    return -8.0 * (1 - x ** 2) ** 3 + 48.0 * x ** 2 * (1 - x ** 2) ** 2


def test_riesz_bump_reduces_to_the_second_derivative_at_alpha_2():
    x = np.linspace(-0.99, 0.99, 41)
    assert np.max(np.abs(O.riesz_bump(x, 2.0) - _bump_second_derivative(x))) <= 1e-11


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_rl_derivative_of_the_bump_matches_its_integral_definition(alpha):
    # f(-1) = f'(-1) = 0, so two integrations by parts of the left Riemann-Liouville derivative
    # (Section 1) give D^alpha f(x) = 1/Gamma(2 - alpha) int_{-1}^x (x - xi)^{1-alpha} f''(xi) dxi;
    # w = (x - xi)^{2-alpha} removes the endpoint singularity before the quadrature
    mpmath.mp.dps = 30
    q = 1.0 / (2.0 - alpha)
    for x in (-0.7, 0.1, 0.85):
        val = mpmath.quad(lambda w: _bump_second_derivative(x - w ** q), [0, (x + 1) ** (2 - alpha)]) * q
        ref = float(val / mpmath.gamma(2 - alpha))
        assert abs(O.rl_left_bump(np.array([x]), alpha)[0] - ref) <= 1e-11 * max(1.0, abs(ref))


def test_fd2_matrix_converges_to_the_riesz_derivative_of_the_bump():
    # D = -h^{-alpha} Toeplitz(g) (eq. FD2) applied to the grid values of f approaches the Riesz
    # derivative at second order away from the boundary: pins the sign and scaling that link the
    # discrete operator to the continuous one
    alpha = 1.5
    errs = []
    for n in (99, 199, 399):
        h = 2.0 / (n + 1)
        x = -1.0 + h * np.arange(1, n + 1)
        D = O.diff_matrix(alpha, n, h)
        inner = np.abs(x) <= 0.5
        errs.append(np.max(np.abs((D @ (1 - x ** 2) ** 4 - O.riesz_bump(x, alpha))[inner])))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


def _printed_errors():
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "example1_printed_errors.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                d, n, steps, err, series = line.split()
                rows.append((int(d), int(n), int(steps), err, series))
    return rows


def _half_unit(printed: str) -> float:
    mant, exp = printed.lower().split("e")
    decimals = len(mant.split(".")[1]) if "." in mant else 0
    return 0.5 * 10.0 ** (int(exp) - decimals)


@pytest.mark.parametrize("steps", [15, 35])
def test_lbdf2_reproduces_the_printed_errors_of_example1_2d(steps):
    row = [r for r in _printed_errors() if r[0] == 2 and r[2] == steps and r[4] == "lbdf2-m"][0]
    params = (1.0, 1.0, 3.0, 1.0, 2.0)
    alpha = (1.2, 1.8)
    U0, src, h = O.example1(row[1], alpha, params)
    P = O.Problem(U0.shape, alpha, h, params, source=src)
    U = O.run(P, "lbdf2", U0, 1.0 / steps, steps)
    err = O.discrete_l2(U - np.exp(-1j) * U0, h)
    assert abs(err - float(row[3])) <= _half_unit(row[3]), (err, row)


def test_strang_reproduces_the_printed_errors_of_example2_2d():
    # the oracle's Strang splitting at n = 800 against the printed errors for 5 and 25 steps,
    # with the reference read as 200 Strang steps (see the fixture)
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "example2_printed_errors.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                d, n, steps, ref_steps, err, _series = line.split()
                if d == "2":
                    rows.append((int(n), int(steps), int(ref_steps), err))
    n = rows[0][0]
    dom = ((-10.0, 10.0),) * 2
    h = [(b - a) / (n + 1) for (a, b) in dom]
    U0 = sech_product(grid_axes((n, n), dom), (1.0, 1.0))
    P = O.Problem((n, n), (1.2, 1.8), h, (1.0, 1.0, 1.0, 1.0, 1.0))
    ref = O.run(P, "strang", U0, 1.0 / rows[0][2], rows[0][2])
    for _, steps, _, printed in (rows[0], rows[-1]):
        err = O.discrete_l2(O.run(P, "strang", U0, 1.0 / steps, steps) - ref, h)
        assert abs(err - float(printed)) <= _half_unit(printed), (steps, err, printed)


@pytest.mark.parametrize("steps", [15, 35])
def test_krogstad_fd4_reproduces_the_printed_errors_of_example1_2d(steps):
    row = [r for r in _printed_errors() if r[4] == "krogstad-m" and r[2] == steps][0]
    params = (1.0, 1.0, 3.0, 1.0, 2.0)
    alpha = (1.2, 1.8)
    U0, src, h = O.example1(row[1], alpha, params)
    P = O.Problem(U0.shape, alpha, h, params, source=src, fd_order=4)
    U = O.run(P, "krogstad", U0, 1.0 / steps, steps)
    err = O.discrete_l2(U - np.exp(-1j) * U0, h)
    assert abs(err - float(row[3])) <= _half_unit(row[3]), (err, row)


def test_krogstad_is_fourth_order_on_the_manufactured_solution():
    P, U0 = _manufactured((10, 12, 8), ((-8.0, 8.0),) * 3, (1.3, 1.6, 1.8))
    T = 0.5
    taus = [0.1, 0.05, 0.025]
    errs = [O.rel_l2(O.run(P, "krogstad", U0, tau, int(round(T / tau))), math.exp(-T) * U0) for tau in taus]
    slopes = np.diff(np.log(errs)) / np.diff(np.log(taus))
    assert abs(slopes[-1] - 4.0) <= 0.2, (errs, slopes)

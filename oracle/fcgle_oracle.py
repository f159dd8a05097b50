"""FP64 CPU oracle for the matrix-/tensor-oriented space-fractional CGLE integrators.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test suite, the smoke check of the entry module
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP library (no kernels, headers, helpers, tables or constant generators).

Everything here is plain numpy/scipy in float64 / complex128, written to be
checked by eye against the paper (Caliari & Cassini, "Matrix- and
tensor-oriented numerical schemes for the evolutionary space-fractional complex
Ginzburg--Landau equation"):

* Section 2: FD2 weights g_k (Gamma form and its stable recurrence), the FD4
  extrapolated weights, the dense Toeplitz matrix D_n^alpha and its
  diagonalisation D = Q Lambda Q^T (LAPACK DSYEV through scipy, then one
  extended-precision orthogonalisation sweep).
* Section 3 (eq. fKu_diag): the Tucker form of f(theta K) v, computed with
  permute-based tensordot mode products.
* Section 3 (eq. Neudeckerd): the exponential as a Kronecker product of 1-D
  exponentials (scipy expm per axis).
* Section 4: the phi-functions (eq. phi), LBDF2 with its backward-forward Euler
  start (eq. lbdf2-v), the pointwise nonlinearity g, and Strang splitting
  (eq. Strang) with the exact flow of the nonlinear subproblem.
* Brute force: K assembled densely as the Kronecker sum (eq. Ksum) for tiny n,
  with expm / solve / augmented-expm for phi_l.

Layout reading: tensors are C-ordered (n_1, ..., n_d) with axis d fastest, so
the C-order vec of U satisfies (M_1 kron ... kron M_d) vec(U) =
vec(U x_1 M_1 ... x_d M_d) and the Kronecker sum is
K = sum_mu I kron ... kron A_mu kron ... kron I with A_1 leftmost.  This is the
paper's operator with the index order relabelled.

Schemes not printed in the paper (exponential Euler, Lawson-Euler, repeated
backward-forward Euler) are written from their textbook definitions; see each
function.  All schemes here are stateless and work in physical space.

Parity status: every function is pinned by the CPU tests (closed forms,
brute force, Neudecker/Sylvester identities, invariants, observed orders,
an adaptive ODE solver for the exact nonlinear flow and for Strang splitting,
the errors the paper prints for its Example 1 (reproduced to all printed digits),
finite differences); none is "parity unpinned".
"""
from __future__ import annotations

import cmath
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

Params = Tuple[float, float, float, float, float]  # (nu, eta, gamma, kappa, zeta)

# ---------------------------------------------------------------------------
# Section 2: spatial semidiscretisation
# ---------------------------------------------------------------------------


def fd2_weights_gamma(alpha: float, n: int) -> np.ndarray:
    """g_k = (-1)^k Gamma(alpha+1) / (Gamma(alpha/2 - k + 1) Gamma(alpha/2 + k + 1)), k = 0..n-1.

    The defining (Gamma) form of the centred fractional difference weights
    (Section 2).  Overflows for large k; used only to pin the recurrence.
    """
    return np.array([(-1) ** k * math.gamma(alpha + 1)
                     / (math.gamma(alpha / 2 - k + 1) * math.gamma(alpha / 2 + k + 1))
                     for k in range(n)])


def fd2_weights(alpha: float, n: int) -> np.ndarray:
    """Stable recurrence for the same weights (Section 2):
    g_0 = Gamma(alpha+1)/Gamma(alpha/2+1)^2,  g_k = (1 - (alpha+1)/(alpha/2+k)) g_{k-1}."""
    g = np.empty(n)
    g[0] = math.gamma(alpha + 1) / math.gamma(alpha / 2 + 1) ** 2
    for k in range(1, n):
        g[k] = (1.0 - (alpha + 1) / (alpha / 2 + k)) * g[k - 1]
    return g


def fd4_weights(alpha: float, n: int) -> np.ndarray:
    """Fourth-order extrapolated weights (Section 2, eq. FD4):
    4/3 g_k for odd k; 4/3 g_k - (1/3) g_{k/2} / 2^alpha for even k."""
    g = fd2_weights(alpha, n)
    out = 4.0 / 3.0 * g
    for k in range(0, n, 2):
        out[k] -= g[k // 2] / (3.0 * 2.0 ** alpha)
    return out


def diff_matrix(alpha: float, n: int, h: float, fd_order: int = 2) -> np.ndarray:
    """D_n^alpha = -h^{-alpha} * symmetric Toeplitz(g_0, ..., g_{n-1})  (Section 2, eq. Dnalpha)."""
    g = fd2_weights(alpha, n) if fd_order == 2 else fd4_weights(alpha, n)
    return -(h ** -alpha) * sla.toeplitz(g)


def eig(D: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """D = Q diag(lam) Q^T with Q orthogonal (Section 2, eq. diag).

    LAPACK DSYEV (the routine the paper uses, Section 4) through scipy, followed by one
    Newton-Schulz orthogonalisation sweep Q <- Q + Q (I - Q^T Q)/2 in extended precision and
    Rayleigh-quotient eigenvalues lam_k = q_k^T D q_k.  Reading: Section 2 requires Q to be
    orthogonal, and the stateless schemes apply Q f Q^T once per step, so any loss of
    orthogonality left by the FP64 solver (a few 1e-15) would accumulate linearly with the
    number of steps; after the sweep Q^T Q = I to rounding of the final FP64 entries.
    """
    lam, Q = sla.eigh(D, driver="ev")
    X = Q.astype(np.longdouble)
    Dl = D.astype(np.longdouble)
    X = X + 0.5 * (X @ (np.eye(D.shape[0], dtype=np.longdouble) - X.T @ X))
    lam = np.sum(X * (Dl @ X), axis=0)
    return lam.astype(np.float64), X.astype(np.float64)


def setup(n: Sequence[int], alpha: Sequence[float], h: Sequence[float], fd_order: int = 2):
    """Per-axis dense D_mu and their eigenpairs."""
    Ds = [diff_matrix(a, m, hh, fd_order) for a, m, hh in zip(alpha, n, h)]
    eigs = [eig(D) for D in Ds]
    return Ds, [e[1] for e in eigs], [e[0] for e in eigs]


# ---------------------------------------------------------------------------
# phi-functions (Section 4, eq. phi)
# ---------------------------------------------------------------------------

_SERIES_TERMS = 40


def phi(l: int, z) -> np.ndarray:
    """phi_0 = e^z; phi_l(z) = (phi_{l-1}(z) - 1/(l-1)!)/z, phi_l(0) = 1/l!.

    For |z| < 1 the recurrence cancels, so there phi_l is summed from its
    Taylor series sum_{k>=0} z^k/(k+l)! (which follows from the recurrence);
    elsewhere the recurrence is used as printed.
    """
    z = np.asarray(z, dtype=np.complex128)
    if l == 0:
        return np.exp(z)
    out = np.empty_like(z)
    small = np.abs(z) < 1.0
    zs = z[small]
    acc = np.zeros_like(zs)
    for k in range(_SERIES_TERMS - 1, -1, -1):  # Horner on sum z^k/(k+l)!
        acc = acc * zs + 1.0 / math.factorial(k + l)
    out[small] = acc
    zl = z[~small]
    p = np.exp(zl)
    for j in range(1, l + 1):
        p = (p - 1.0 / math.factorial(j - 1)) / zl
    out[~small] = p
    return out


def f_of(kind: str, z) -> np.ndarray:
    """The scalar functions the schemes need: 'inv' -> 1/(1-z), 'exp' -> e^z, 'phiL' -> phi_L."""
    z = np.asarray(z, dtype=np.complex128)
    if kind == "inv":
        return 1.0 / (1.0 - z)
    if kind == "exp":
        return np.exp(z)
    if kind.startswith("phi"):
        return phi(int(kind[3:]), z)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Section 3: mode products and the Tucker operator
# ---------------------------------------------------------------------------


def mode_product(U: np.ndarray, M: np.ndarray, mu: int) -> np.ndarray:
    """U x_mu M: multiply M onto the mode-mu fibres of U (Section 3).

    out[..., i, ...] = sum_k M[i, k] U[..., k, ...] along axis mu, done by
    tensordot + moveaxis (i.e. with a permutation).  A real M is applied to the
    real and imaginary parts separately.
    """
    if np.isrealobj(M) and np.iscomplexobj(U):
        re = np.moveaxis(np.tensordot(M, U.real, axes=([1], [mu])), 0, mu)
        im = np.moveaxis(np.tensordot(M, U.imag, axes=([1], [mu])), 0, mu)
        return re + 1j * im
    return np.moveaxis(np.tensordot(M, U, axes=([1], [mu])), 0, mu)


def tucker(U: np.ndarray, Ms: Sequence[np.ndarray]) -> np.ndarray:
    """U x_1 M_1 x_2 ... x_d M_d."""
    out = U
    for mu, M in enumerate(Ms):
        out = mode_product(out, M, mu)
    return out


def ell_grid(lams: Sequence[np.ndarray]) -> np.ndarray:
    """ell_{j_1..j_d} = sum_mu lambda^{(mu)}_{j_mu}: eigenvalues of D_1 (+) ... (+) D_d."""
    d = len(lams)
    ell = np.zeros([len(l) for l in lams])
    for mu, lam in enumerate(lams):
        shape = [1] * d
        shape[mu] = len(lam)
        ell = ell + lam.reshape(shape)
    return ell


def f_grid(kind: str, theta: float, lams: Sequence[np.ndarray], params: Params) -> np.ndarray:
    """F = f(theta (nu + i eta) ell) collected on the grid (Section 3)."""
    nu, eta = params[0], params[1]
    return f_of(kind, theta * (nu + 1j * eta) * ell_grid(lams))


def apply_f(kind: str, theta: float, V: np.ndarray, Qs, lams, params: Params) -> np.ndarray:
    """f(theta K) v = vec(((F o (V x_mu Q_mu^T)) x_mu Q_mu))  (Section 3, eq. fKu_diag)."""
    Vhat = tucker(V, [Q.T for Q in Qs])
    return tucker(f_grid(kind, theta, lams, params) * Vhat, Qs)


def apply_K(U: np.ndarray, Ds: Sequence[np.ndarray], params: Params) -> np.ndarray:
    """K u = vec(sum_mu U x_mu A_mu), A_mu = (nu + i eta) D_mu, with dense D (Section 3, eq. kronsumv)."""
    c = params[0] + 1j * params[1]
    out = np.zeros_like(U, dtype=np.complex128)
    for mu, D in enumerate(Ds):
        out = out + mode_product(U, D, mu)
    return c * out


def exp_neudecker(theta: float, V: np.ndarray, Ds: Sequence[np.ndarray], params: Params) -> np.ndarray:
    """exp(theta K) v = vec(V x_1 exp(theta A_1) ... x_d exp(theta A_d))  (Section 3, eq. Neudeckerd)."""
    c = params[0] + 1j * params[1]
    return tucker(V.astype(np.complex128), [sla.expm(theta * c * D) for D in Ds])


# ---------------------------------------------------------------------------
# Brute force on the assembled Kronecker sum (tiny n only)
# ---------------------------------------------------------------------------


def kron_sum(Ds: Sequence[np.ndarray], params: Params) -> np.ndarray:
    """Dense K = sum_mu I kron ... kron A_mu kron ... kron I in C-order (A_1 leftmost)."""
    c = params[0] + 1j * params[1]
    sizes = [D.shape[0] for D in Ds]
    N = int(np.prod(sizes))
    K = np.zeros((N, N), np.complex128)
    for mu, D in enumerate(Ds):
        term = np.ones((1, 1))
        for nu_, m in enumerate(sizes):
            term = np.kron(term, c * D if nu_ == mu else np.eye(m))
        K = K + term
    return K


def brute_apply(kind: str, theta: float, V: np.ndarray, Ds, params: Params) -> np.ndarray:
    """f(theta K) v with K assembled: expm, solve(I - theta K, v), or phi_l through the
    augmented-matrix exponential exp([[theta K, v e_1^T], [0, J]]) whose last block column
    holds phi_1(theta K) v, ..., phi_l(theta K) v (J the l x l upper shift)."""
    K = kron_sum(Ds, params)
    v = V.reshape(-1).astype(np.complex128)
    N = v.size
    A = theta * K
    if kind == "exp":
        out = sla.expm(A) @ v
    elif kind == "inv":
        out = np.linalg.solve(np.eye(N) - A, v)
    elif kind.startswith("phi"):
        l = int(kind[3:])
        W = np.zeros((N + l, N + l), np.complex128)
        W[:N, :N] = A
        W[:N, N] = v
        for j in range(l - 1):
            W[N + j, N + j + 1] = 1.0
        out = sla.expm(W)[:N, N + l - 1]
    else:
        raise ValueError(kind)
    return out.reshape(V.shape)


# ---------------------------------------------------------------------------
# Nonlinearity and source (Section 2)
# ---------------------------------------------------------------------------


class Source:
    """s(t) = sum_k exp(rate_k t) S_k with real or complex rates (zero when there are no terms)."""

    def __init__(self, rates: Sequence[complex] = (), tensors: Sequence[np.ndarray] = ()):
        self.rates = list(rates)
        self.tensors = list(tensors)

    def __call__(self, t: float, shape) -> np.ndarray:
        s = np.zeros(shape, np.complex128)
        for r, S in zip(self.rates, self.tensors):
            s = s + cmath.exp(r * t) * S
        return s


def g_nonlin(t: float, U: np.ndarray, params: Params, source: Optional[Source] = None) -> np.ndarray:
    """g(t, u)_j = gamma u_j - (kappa + i zeta) |u_j|^2 u_j + s(t, x_j)  (Section 2)."""
    _, _, gamma, kappa, zeta = params
    out = gamma * U - (kappa + 1j * zeta) * (np.abs(U) ** 2) * U
    if source is not None:
        out = out + source(t, U.shape)
    return out


def manufactured_source(U0: np.ndarray, Ds, params: Params) -> Source:
    """Semi-discrete source making u(t) = e^{-t} U0 the exact solution of u' = K u + g(t, u):
    s(t) = e^{-t} (-(1 + gamma) U0 - K U0) + e^{-3t} (kappa + i zeta) |U0|^2 U0,
    with K U0 formed by dense mode products (Section 3, eq. kronsumv)."""
    _, _, gamma, kappa, zeta = params
    S1 = -(1.0 + gamma) * U0 - apply_K(U0, Ds, params)
    S3 = (kappa + 1j * zeta) * (np.abs(U0) ** 2) * U0
    return Source((-1.0, -3.0), (S1, S3))


# ---------------------------------------------------------------------------
# The paper's Example 1 (Section 4): exact solution e^{-it} prod_mu (1 - x_mu^2)^4
# ---------------------------------------------------------------------------


def rl_left_bump(x, alpha: float) -> np.ndarray:
    """Left Riemann-Liouville derivative from -1 (Section 1) of f(x) = (1 - x^2)^4 on (-1, 1)
    (f extended by zero outside).  Writing 1 - x = 2 - (1 + x),
    f = sum_{k=0..4} C(4,k) 2^{4-k} (-1)^k (1 + x)^{4+k}, and each power has
    D^alpha (1 + x)^p = Gamma(p + 1) / Gamma(p + 1 - alpha) (1 + x)^{p - alpha}."""
    from scipy.special import gamma as Gam
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for k in range(5):
        p = 4 + k
        c = math.comb(4, k) * 2.0 ** (4 - k) * (-1.0) ** k
        out = out + c * Gam(p + 1.0) / Gam(p + 1.0 - alpha) * (1.0 + x) ** (p - alpha)
    return out


def riesz_bump(x, alpha: float) -> np.ndarray:
    """Riesz derivative of f(x) = (1 - x^2)^4 (Section 1): -(D_left f + D_right f)/(2 cos(alpha pi/2)).
    f is even, so its right Riemann-Liouville derivative at x is the left one at -x."""
    x = np.asarray(x, dtype=np.float64)
    return -(rl_left_bump(x, alpha) + rl_left_bump(-x, alpha)) / (2.0 * math.cos(alpha * math.pi / 2.0))


def example1(n: int, alpha: Sequence[float], params: Params):
    """The paper's Example 1 (Section 4) on (-1,1)^d, n inner points per axis (h = 2/(n+1)):
    u(t, x) = e^{-it} F(x), F = prod_mu (1 - x_mu^2)^4, solves eq. FCGLE with the source
    s = u_t - (nu + i eta) sum_mu d^{alpha_mu} u - gamma u + (kappa + i zeta)|u|^2 u = e^{-it} S,
    S = -i F - (nu + i eta) sum_mu R_mu F - gamma F + (kappa + i zeta) F^3  (F real and |e^{-it}| = 1,
    R_mu the Riesz derivative along axis mu).  Returns (U0 = F, Source with rate -i, h)."""
    nu, eta, gamma, kappa, zeta = params
    d = len(alpha)
    h = 2.0 / (n + 1)
    x = -1.0 + h * np.arange(1, n + 1)
    f = (1.0 - x ** 2) ** 4

    def outer(vs):
        out = vs[0]
        for v in vs[1:]:
            out = np.multiply.outer(out, v)
        return out

    F = outer([f] * d)
    RF = np.zeros_like(F)
    for mu in range(d):
        RF = RF + outer([riesz_bump(x, alpha[mu]) if nu_ == mu else f for nu_ in range(d)])
    S = -1j * F - (nu + 1j * eta) * RF - gamma * F + (kappa + 1j * zeta) * F ** 3
    return F.astype(np.complex128), Source((-1j,), (S,)), (h,) * d


def discrete_l2(E: np.ndarray, h: Sequence[float]) -> float:
    """(prod_mu h_mu sum_j |E_j|^2)^{1/2}, the discrete L2 norm of the paper's absolute errors."""
    return math.sqrt(float(np.prod(h)) * float(np.sum(np.abs(E) ** 2)))


# ---------------------------------------------------------------------------
# Time schemes (stateless, physical space)
# ---------------------------------------------------------------------------


class Problem:
    """Bundle of the semidiscrete problem: eigenpairs, parameters and source."""

    def __init__(self, n, alpha, h, params: Params, source: Optional[Source] = None, fd_order: int = 2):
        self.n = tuple(int(m) for m in n)
        self.params = tuple(float(p) for p in params)
        self.Ds, self.Qs, self.lams = setup(n, alpha, h, fd_order)
        self.source = source

    def f(self, kind: str, theta: float, V: np.ndarray) -> np.ndarray:
        return apply_f(kind, theta, V, self.Qs, self.lams, self.params)

    def g(self, t: float, U: np.ndarray) -> np.ndarray:
        return g_nonlin(t, U, self.params, self.source)


def step_exp_euler(P: Problem, U: np.ndarray, t: float, tau: float) -> np.ndarray:
    """Exponential Euler: u_{n+1} = e^{tau K} u_n + tau phi_1(tau K) g(t_n, u_n).
    (The first stage of the paper's Krogstad scheme, Section 4, taken with step tau.)"""
    return P.f("exp", tau, U) + tau * P.f("phi1", tau, P.g(t, U))


def step_lawson(P: Problem, U: np.ndarray, t: float, tau: float) -> np.ndarray:
    """Lawson-Euler: u_{n+1} = e^{tau K} (u_n + tau g(t_n, u_n))."""
    return P.f("exp", tau, U + tau * P.g(t, U))


def step_bfe(P: Problem, U: np.ndarray, t: float, tau: float) -> np.ndarray:
    """Backward-forward Euler (the paper's LBDF2 start, Section 4):
    (I - tau K) u_{n+1} = u_n + tau g(t_n, u_n)."""
    return P.f("inv", tau, U + tau * P.g(t, U))


def step_lbdf2(P: Problem, U: np.ndarray, Uprev: np.ndarray, t: float, tau: float) -> np.ndarray:
    """Linearised BDF2 (Section 4, eq. lbdf2-v), t = t_n:
    (I - 2tau/3 K) u_{n+1} = 4/3 u_n - 1/3 u_{n-1} + 2tau/3 g(t_{n+1}, 2 u_n - u_{n-1})."""
    rhs = (4.0 / 3.0) * U - (1.0 / 3.0) * Uprev + (2.0 * tau / 3.0) * P.g(t + tau, 2.0 * U - Uprev)
    return P.f("inv", 2.0 * tau / 3.0, rhs)


def step_krogstad(P: Problem, U: np.ndarray, t: float, tau: float) -> np.ndarray:
    """Krogstad's fourth-order exponential Runge-Kutta step (Section 4, eq. krogstad-v):
    f_n = K u_n + g(t_n, u_n), d_i = g(t_n + c_i tau, u_{ni}) - g(t_n, u_n), c_2 = c_3 = 1/2, c_4 = 1,
        u_{n2}  = u_n + tau/2 phi_1(tau/2 K) f_n
        u_{n3}  = u_n + tau/2 phi_1(tau/2 K) f_n + tau phi_2(tau/2 K) d_2
        u_{n4}  = u_n + tau phi_1(tau K) f_n + 2 tau phi_2(tau K) d_3
        u_{n+1} = u_n + tau phi_1(tau K) f_n + tau phi_2(tau K)(2 d_2 + 2 d_3 - d_4)
                  + tau phi_3(tau K)(-4 d_2 - 4 d_3 + 4 d_4),
    with K u_n formed by dense mode products with the D_mu (eq. kronsumv)."""
    g_n = P.g(t, U)
    f_n = apply_K(U, P.Ds, P.params) + g_n
    half = U + 0.5 * tau * P.f("phi1", 0.5 * tau, f_n)
    d2 = P.g(t + 0.5 * tau, half) - g_n
    u3 = half + tau * P.f("phi2", 0.5 * tau, d2)
    d3 = P.g(t + 0.5 * tau, u3) - g_n
    full = U + tau * P.f("phi1", tau, f_n)
    u4 = full + 2.0 * tau * P.f("phi2", tau, d3)
    d4 = P.g(t + tau, u4) - g_n
    return (full + tau * P.f("phi2", tau, 2.0 * d2 + 2.0 * d3 - d4)
            + tau * P.f("phi3", tau, -4.0 * d2 - 4.0 * d3 + 4.0 * d4))


def nonlinear_flow(W: np.ndarray, t: float, params: Params) -> np.ndarray:
    """Exact flow phi_t of the nonlinear subproblem w' = gamma w - (kappa + i zeta)|w|^2 w
    (Section 4, Strang splitting):
        phi_t(w0) = exp(t gamma - (kappa + i zeta)/(2 kappa) log(1 + 2 t phi_1(2 gamma t) kappa |w0|^2)) w0.
    For kappa = 0 the exponent is its limit kappa -> 0, t gamma - i zeta t phi_1(2 gamma t) |w0|^2."""
    _, _, gamma, kappa, zeta = params
    W = np.asarray(W, dtype=np.complex128)
    tp1 = t * phi(1, np.array([2.0 * gamma * t])).real[0]  # t phi_1(2 gamma t)
    m = np.abs(W) ** 2
    if kappa > 0.0:
        expo = t * gamma - (kappa + 1j * zeta) / (2.0 * kappa) * np.log(1.0 + 2.0 * tp1 * kappa * m)
    else:
        expo = t * gamma - 1j * zeta * tp1 * m
    return np.exp(expo) * W


def step_strang(P: Problem, U: np.ndarray, t: float, tau: float) -> np.ndarray:
    """Strang splitting (Section 4, eq. Strang): u_{n+1} = phi_{tau/2}(e^{tau K} phi_{tau/2}(u_n)).
    The nonlinear flow is exact only for the autonomous nonlinearity, so a source is rejected."""
    if P.source is not None and P.source.rates:
        raise ValueError("Strang splitting takes no source term")
    half = nonlinear_flow(U, 0.5 * tau, P.params)
    return nonlinear_flow(P.f("exp", tau, half), 0.5 * tau, P.params)


def run(P: Problem, scheme: str, U0: np.ndarray, tau: float, steps: int, t0: float = 0.0,
        callback: Optional[Callable[[int, np.ndarray], None]] = None) -> np.ndarray:
    """March `steps` steps of `scheme` in {'exp_euler', 'lawson', 'lie', 'lbdf2', 'strang', 'krogstad'} from
    U0 at t0.  'lie' repeats the backward-forward Euler step; 'lbdf2' starts with one such step."""
    U = U0.astype(np.complex128)
    Uprev = None
    t = t0
    for k in range(steps):
        if scheme == "exp_euler":
            Un = step_exp_euler(P, U, t, tau)
        elif scheme == "lawson":
            Un = step_lawson(P, U, t, tau)
        elif scheme == "lie":
            Un = step_bfe(P, U, t, tau)
        elif scheme == "lbdf2":
            Un = step_bfe(P, U, t, tau) if Uprev is None else step_lbdf2(P, U, Uprev, t, tau)
        elif scheme == "strang":
            Un = step_strang(P, U, t, tau)
        elif scheme == "krogstad":
            Un = step_krogstad(P, U, t, tau)
        else:
            raise ValueError(scheme)
        Uprev, U = U, Un
        t = t0 + (k + 1) * tau
        if callback is not None:
            callback(k + 1, U)
    return U


# ---------------------------------------------------------------------------
# Discrete adjoint of exponential Euler
# ---------------------------------------------------------------------------


def expeuler_vjp(P: Problem, U: np.ndarray, Ubar_next: np.ndarray, t: float, tau: float):
    """Vector-Jacobian product of one exponential-Euler step u_{n+1} = E u_n + tau P1 g(t_n, u_n),
    E = e^{tau K}, P1 = phi_1(tau K), for a real loss with cotangent convention
    ubar = dL/dRe(u) + i dL/dIm(u).

    E and P1 are complex symmetric (Q real orthogonal), so their adjoints are the
    same functions of the conjugated eigenvalues:
      w       = tau phi_1(tau K)^H ubar_{n+1}
      ubar_n  = e^{tau K}^H ubar_{n+1} + (gamma - 2 conj(c) |u_n|^2) w - c u_n^2 conj(w),  c = kappa + i zeta
    Parameter cotangents (source independent of parameters):
      gamma: Re sum conj(w) u_n;  kappa: Re sum conj(w)(-|u|^2 u);  zeta: Re sum conj(w)(-i |u|^2 u)
      nu, eta: Re sum conj(a) * dz * (e^z b + tau phi_1'(z) ghat) with a = Q^T ubar_{n+1},
      b = Q^T u_n, ghat = Q^T g_n, dz = tau ell (nu) or i tau ell (eta), phi_1' = phi_1 - phi_2.
    Returns (ubar_n, pbar) with pbar ordered (nu, eta, gamma, kappa, zeta).
    """
    nu, eta, gamma, kappa, zeta = P.params
    c = kappa + 1j * zeta
    ell = ell_grid(P.lams)
    z = tau * (nu + 1j * eta) * ell
    QT = [Q.T for Q in P.Qs]
    a_hat = tucker(Ubar_next, QT)
    lin = tucker(np.conj(np.exp(z)) * a_hat, P.Qs)
    w = tau * tucker(np.conj(phi(1, z)) * a_hat, P.Qs)
    absu2 = np.abs(U) ** 2
    ubar = lin + (gamma - 2.0 * np.conj(c) * absu2) * w - c * U * U * np.conj(w)
    gn = P.g(t, U)
    b_hat = tucker(U, QT)
    g_hat = tucker(gn, QT)
    X = np.exp(z) * b_hat + tau * (phi(1, z) - phi(2, z)) * g_hat
    nubar = np.real(np.sum(np.conj(a_hat) * tau * ell * X))
    etabar = np.real(np.sum(np.conj(a_hat) * 1j * tau * ell * X))
    gbar = np.real(np.sum(np.conj(w) * U))
    kbar = np.real(np.sum(np.conj(w) * (-absu2 * U)))
    zbar = np.real(np.sum(np.conj(w) * (-1j * absu2 * U)))
    return ubar, np.array([nubar, etabar, gbar, kbar, zbar])


def expeuler_loss_and_grad(P: Problem, U0: np.ndarray, Utarget: np.ndarray, tau: float, steps: int,
                           t0: float = 0.0):
    """L = ||u(T) - u_target||^2 (plain sum of squares) after `steps` exponential-Euler steps,
    with its gradient w.r.t. u0 (same convention as expeuler_vjp) and the five parameters,
    by storing the forward trajectory and sweeping the step adjoint backwards."""
    traj = [U0.astype(np.complex128)]
    U = traj[0]
    for k in range(steps):
        U = step_exp_euler(P, U, t0 + k * tau, tau)
        traj.append(U)
    diff = U - Utarget
    L = float(np.sum(np.abs(diff) ** 2))
    ubar = 2.0 * diff
    pbar = np.zeros(5)
    for k in range(steps - 1, -1, -1):
        ubar, pb = expeuler_vjp(P, traj[k], ubar, t0 + k * tau, tau)
        pbar += pb
    return L, ubar, pbar


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 (the h-weights of the discrete L2 norm cancel)."""
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))

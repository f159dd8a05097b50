"""GPU parity of the refined inverse (fcgle_apply_inv_refined) against the FP64 oracle.

x = (I - theta (nu + i eta) K)^{-1} v: the reduced-precision inverse (FP32 MFMA or split
BF16) followed by refinement sweeps whose residual is formed in FP64 with the Toeplitz D_mu.
Bar: relative L2 error against the oracle's inverse <= 1e-12 after the stated number of
sweeps for every precision; the reported residual norms decrease and the last one equals the
oracle's residual of the returned x.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fcgle_oracle as O
from workloads import random_complex

pytestmark = pytest.mark.gpu

# sweeps after which the refined inverse is at FP64 accuracy: a sweep multiplies the error by
# about (operator error of the precision) x cond(I - theta (nu + i eta) K), i.e. ~1e-16 / 1e-5 /
# 1e-5 / 1e-3 for the FP64 / FP32 / split-BF16x6 / split-BF16x3 inverse at these theta
SWEEPS = {"fp64": 1, "fp32": 2, "bf16x6": 2, "bf16x3": 3}
TOL0 = {"fp64": 1e-12, "fp32": 1e-5, "bf16x6": 1e-5, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def F():
    import paper_2510_21394_amd as pkg
    return pkg


def _setup(n, seed):
    rng = np.random.default_rng(seed)
    return tuple(rng.uniform(1.15, 1.95, len(n))), tuple(rng.uniform(0.05, 0.4, len(n)))


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


def _residual(P, theta, V, X):
    """||v - (I - theta (nu + i eta) K) x|| / ||v|| with the oracle's K (dense D_mu)."""
    R = V - X + theta * O.apply_K(X, P.Ds, P.params)
    return float(np.linalg.norm(R) / np.linalg.norm(V))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("n", [(20, 33, 17), (130, 75), (300,), (5, 6, 7, 8)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("theta", [1e-2, 0.1])
def test_refined_inverse_matches_oracle(F, prec, n, theta):
    alpha, h = _setup(n, 61 + len(n))
    params = (0.8, -0.6, 1.0, 1.0, 0.5)
    V = random_complex(n, 62)
    P = O.Problem(n, alpha, h, params)
    ref = P.f("inv", theta, V)
    plan = F.Plan(n, alpha, h, params, tau=1e-3, precision=prec)
    v = torch.from_numpy(V).cuda()
    x0, r0 = plan.apply_inv_refined(theta, v, sweeps=0, residuals=True)
    e0 = O.rel_l2(_host(x0), ref)
    s = SWEEPS[prec]
    x, rn = plan.apply_inv_refined(theta, v, sweeps=s, residuals=True)
    e = O.rel_l2(_host(x), ref)
    print(f"[refine {prec} {n} theta={theta}] rel_l2 sweeps=0: {e0:.3e}, sweeps={s}: {e:.3e}; residuals {rn}")
    assert e0 <= TOL0[prec]
    assert e <= 1e-12
    assert len(rn) == s + 1 and abs(rn[0] - r0[0]) <= 1e-6 * max(r0[0], 1e-30)
    for a, b in zip(rn, rn[1:]):
        assert b <= a or b <= 1e-14
    assert abs(rn[-1] - _residual(P, theta, V, _host(x))) <= 1e-3 * rn[-1] + 1e-15
    torch.testing.assert_close(v, torch.from_numpy(V).cuda(), rtol=0, atol=0)  # v is read only
    plan.close()


def test_refined_inverse_argument_errors(F):
    n = (8, 9)
    alpha, h = _setup(n, 7)
    plan = F.Plan(n, alpha, h, (1.0, 0.5, 1.0, 1.0, 0.5), tau=1e-3, precision="fp32")
    v = torch.from_numpy(random_complex(n, 3)).cuda()
    with pytest.raises(F.FcgleError):
        plan.apply_inv_refined(0.1, v, sweeps=1, out=v)
    with pytest.raises(F.FcgleError):
        plan.apply_inv_refined(0.1, v, sweeps=9)
    with pytest.raises(ValueError):
        plan.apply_inv_refined(0.1, v.to(torch.complex64), sweeps=1)
    x = plan.apply_inv_refined(0.1, v, sweeps=2)
    assert torch.isfinite(torch.view_as_real(x)).all()
    plan.close()

"""GPU tests of the two tensor loaders of the mode products: per-k-tile buffer views with
32-bit offsets (the default) and 64-bit element indices (the WIDE tile configurations, which
the library takes for N-loader products whose 32 rows span more than 2 GiB).

Small shapes: the 64-bit loader, forced on every N-loader product, against the FP64 oracle at
the parity tests' tolerances and against the default loader.  Full stride: tensors whose
axis-0 products need the 64-bit loader, checked by a property that holds at any size (Section
3): a Kronecker product v of eigenvectors of the D_mu is an eigenvector of every f(theta K),
f(theta K) v = f(theta (nu + i eta) sum_mu lambda_mu) v, so the output must be that multiple
of the input element by element.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fcgle_oracle as O
from workloads import random_complex

pytestmark = pytest.mark.gpu

TOL_OP = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4, "bf16x6": 1e-5}
CDT = {"fp64": torch.complex128, "fp32": torch.complex64, "bf16x3": torch.complex64, "bf16x6": torch.complex64}
PARAMS = (0.8, -0.6, 1.0, 1.0, 0.5)


@pytest.fixture(scope="module")
def F():
    import paper_2510_21394_amd as pkg
    return pkg


def _dev(x, prec):
    return torch.from_numpy(np.ascontiguousarray(x)).to(CDT[prec]).cuda()


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("n", [(130, 75), (20, 33, 17), (5, 6, 7, 8)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("split", [True, False], ids=["evenodd", "dense"])
def test_forced_64bit_loads_match_oracle(F, prec, n, split):
    rng = np.random.default_rng(3 + len(n))
    alpha = tuple(rng.uniform(1.15, 1.95, len(n)))
    h = tuple(rng.uniform(0.05, 0.4, len(n)))
    V = random_complex(n, 11)
    P = O.Problem(n, alpha, h, PARAMS)
    plan = F.Plan(n, alpha, h, PARAMS, tau=1e-3, precision=prec)
    plan.set_structure(split)
    for kind in ("exp", "inv"):
        ref = P.f(kind, 1e-2, V)
        base = _host(plan.apply_f(kind, 1e-2, _dev(V, prec)))
        plan.set_wide_loads(True)
        assert "loads=64-bit-index(axes " + ",".join(str(m) for m in range(len(n) - 1)) + ")" in plan.describe()
        wide = _host(plan.apply_f(kind, 1e-2, _dev(V, prec)))
        plan.set_wide_loads(False)
        assert "loads=64-bit-index" not in plan.describe()
        print(f"[{prec} {n} split={split} {kind}] oracle {_rel(wide, ref):.3e}, default loader {_rel(wide, base):.3e}")
        assert _rel(wide, ref) <= TOL_OP[prec]
        assert _rel(wide, base) <= TOL_OP[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forced_64bit_loads_exp_euler_run(F, prec):
    n = (20, 33, 17)
    alpha, h = (1.3, 1.7, 1.5), (0.2, 0.1, 0.3)
    U0 = random_complex(n, 5) * 0.5
    tau, steps = 1e-3, 6
    ref = O.run(O.Problem(n, alpha, h, PARAMS), "exp_euler", U0, tau, steps)
    plan = F.Plan(n, alpha, h, PARAMS, tau=tau, precision=prec)
    plan.set_fusion(True, True, False, update_in_backward=True, phi1_on_the_fly=True)
    plan.set_wide_loads(True)
    u = _dev(U0, prec)
    plan.run("exp_euler", u, 0.0, steps)
    err = _rel(_host(u), ref)
    print(f"[exp_euler {prec} 64-bit loads] rel_l2 = {err:.3e}")
    assert err <= TOL_OP[prec]
    plan.close()


# (shape, precision, tolerance): 4-D tensors whose axis-0 stride B = n_1 n_2 n_3 needs the 64-bit
# loader (32 B sizeof(complex) > 2^31: B > 2^23 for complex64, 2^22 for complex128) while the
# axes stay short enough for a quick set-up.
WIDE_CASES = [((3, 290, 200, 150), "fp32", 1e-4), ((3, 210, 150, 140), "fp64", 1e-11)]


@pytest.mark.parametrize("n,prec,tol", WIDE_CASES, ids=["fp32-3x290x200x150", "fp64-3x210x150x140"])
def test_wide_stride_eigenvector_property(F, n, prec, tol):
    d = len(n)
    alpha, h = (1.5, 1.4, 1.6, 1.3), (0.2, 0.02, 0.03, 0.025)
    theta = 1e-3
    plan = F.Plan(n, alpha, h, PARAMS, tau=1e-3, precision=prec)
    desc = plan.describe()
    print(desc)
    assert "loads=64-bit-index(axes 0)" in desc
    eig = [plan.eig(mu) for mu in range(d)]
    nu, eta = PARAMS[0], PARAMS[1]
    for idx in (tuple(m - 1 for m in n), (0, n[1] // 2, 3, n[3] - 7)):
        q = [eig[mu][0][:, idx[mu]] for mu in range(d)]
        lam = sum(eig[mu][1][idx[mu]] for mu in range(d))
        v = np.einsum("i,j,k,l->ijkl", *q)
        scale = np.exp(theta * (nu + 1j * eta) * lam)
        for kind, f in (("exp", scale), ("inv", 1.0 / (1.0 - theta * (nu + 1j * eta) * lam))):
            out = _host(plan.apply_f(kind, theta, _dev(v, prec)))
            err = _rel(out, f * v)
            print(f"[{prec} {n} eigvec {idx} {kind}] |f| = {abs(f):.4f}, rel_l2 = {err:.3e}")
            assert err <= tol
    plan.close()

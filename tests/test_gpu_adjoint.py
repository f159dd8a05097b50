"""GPU parity of the exponential-Euler adjoint (fcgle_vjp / fcgle_vjp_run and the autograd
trajectory with checkpoints) against the FP64 oracle's discrete adjoint.

Tolerances (relative L2 over the whole cotangent; parameter cotangents relative to their
vector norm): FP64 <= 1e-10 (the two sides differ only by rounding order and by the
library's recomputation of the segment from its checkpoint); FP32 <= 1e-4.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fcgle_oracle as O
from workloads import (ADJOINT_CHECKPOINT_EVERY, ADJOINT_PERTURBATION, BASE_PARAMS, adjoint_3d, grid_axes,
                       random_complex, sech_product, u0_adjoint)

pytestmark = pytest.mark.gpu

CDT = {"fp64": torch.complex128, "fp32": torch.complex64}
TOL = {"fp64": 1e-10, "fp32": 1e-4}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "3d_96_adjoint.npz")


@pytest.fixture(scope="module")
def F():
    import paper_2510_21394_amd as pkg
    return pkg


def _dev(x, prec):
    return torch.from_numpy(np.ascontiguousarray(x)).to(CDT[prec]).cuda()


def _host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    dom = ((-10.0, 10.0),) * len(n)
    alpha = tuple(rng.uniform(1.2, 1.9, len(n)))
    h = [(b - a) / (m + 1) for (a, b), m in zip(dom, n)]
    return dom, alpha, h


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [(20, 33, 17), (40, 27)], ids=lambda s: "x".join(map(str, s)))
def test_single_step_vjp_matches_oracle(F, prec, n):
    dom, alpha, h = _problem(n, 11)
    params = (0.9, -0.4, 0.7, 1.3, 0.6)
    tau, t = 2e-3, 0.1
    U = 1.5 * sech_product(grid_axes(n, dom), [0.5] + [0.3] * (len(n) - 1), 0.2) + 0.1 * random_complex(n, 3)
    Ubar = random_complex(n, 4)
    P = O.Problem(n, alpha, h, params)
    ref_u, ref_p = O.expeuler_vjp(P, U, Ubar, t, tau)
    plan = F.Plan(n, alpha, h, params, tau=tau, precision=prec)
    pbar = torch.zeros(5, dtype=torch.float64, device="cuda")
    out = plan.vjp(_dev(U, prec), _dev(Ubar, prec), t, pbar)
    eu = _rel(_host(out), ref_u)
    ep = float(np.linalg.norm(pbar.cpu().numpy() - ref_p) / np.linalg.norm(ref_p))
    print(f"[vjp {prec} {n}] ubar rel_l2 = {eu:.3e}, pbar rel = {ep:.3e}")
    assert eu <= TOL[prec]
    assert ep <= TOL[prec]
    plan.close()


def test_vjp_in_place_and_accumulating(F):
    n = (12, 10, 14)
    dom, alpha, h = _problem(n, 5)
    params = BASE_PARAMS
    tau = 1e-3
    U = sech_product(grid_axes(n, dom), [1.0, 0.0, 0.0])
    Ubar = random_complex(n, 8)
    P = O.Problem(n, alpha, h, params)
    ref_u, ref_p = O.expeuler_vjp(P, U, Ubar, 0.0, tau)
    plan = F.Plan(n, alpha, h, params, tau=tau, precision="fp64")
    pbar = torch.full((5,), 1.0, dtype=torch.float64, device="cuda")  # added to, not overwritten
    ub = _dev(Ubar, "fp64")
    plan.vjp(_dev(U, "fp64"), ub, 0.0, pbar, ubar_n=ub)
    assert _rel(_host(ub), ref_u) <= 1e-10
    np.testing.assert_allclose(pbar.cpu().numpy(), ref_p + 1.0, rtol=1e-10, atol=1e-12)
    with pytest.raises(F.FcgleError):
        plan.vjp(ub, ub, 0.0, pbar)  # u_n aliasing the cotangent
    plan.close()


def test_vjp_rejects_other_schemes(F):
    n = (8, 9)
    dom, alpha, h = _problem(n, 2)
    plan = F.Plan(n, alpha, h, BASE_PARAMS, tau=1e-3, precision="fp64")
    u = _dev(random_complex(n, 1), "fp64")
    pbar = torch.zeros(5, dtype=torch.float64, device="cuda")
    for scheme in ("lawson", "lie", "lbdf2"):
        with pytest.raises(F.FcgleError) as e:
            plan.vjp(u, u.clone(), 0.0, pbar, scheme=scheme)
        assert e.value.code == -2
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpointed_gradient_matches_oracle(F, prec):
    """Loss ||u(T) - u_target||^2 after 23 steps with checkpoints every 5 steps (a ragged last
    segment): gradient w.r.t. u0 and the five parameters vs the oracle's stored-trajectory adjoint."""
    n = (16, 20, 12)
    dom, alpha, h = _problem(n, 21)
    params = (1.0, 0.5, 1.0, 1.0, 0.5)
    tau, steps, every = 1e-3, 23, 5
    U0 = sech_product(grid_axes(n, dom), [1.0, 0.0, 0.0]) * 1.2
    Ut = 0.8 * sech_product(grid_axes(n, dom), [0.7, 0.2, 0.0], 0.3)
    P = O.Problem(n, alpha, h, params)
    Lref, gref, pref = O.expeuler_loss_and_grad(P, U0, Ut, tau, steps)

    prob = F.Problem(n, alpha, h, tau=tau, precision=prec)
    u0 = _dev(U0, prec).requires_grad_(True)
    pt = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    uT = prob.trajectory(u0, pt, steps, every=every)
    loss = (uT - _dev(Ut, prec)).abs().pow(2).sum()
    loss.backward()
    eu = _rel(_host(u0.grad), gref)
    ep = float(np.linalg.norm(pt.grad.numpy() - pref) / np.linalg.norm(pref))
    el = abs(float(loss) - Lref) / Lref
    print(f"[grad {prec} {n} x{steps}/{every}] u0 rel_l2 = {eu:.3e}, params rel = {ep:.3e}, loss rel = {el:.3e}")
    assert eu <= TOL[prec]
    assert ep <= TOL[prec]
    assert el <= TOL[prec]
    prob.close()


def test_checkpoint_interval_does_not_change_the_gradient(F):
    n = (18, 14, 10)
    dom, alpha, h = _problem(n, 9)
    tau, steps = 1e-3, 12
    U0 = sech_product(grid_axes(n, dom), [1.0, 0.0, 0.0])
    Ut = random_complex(n, 12) * 0.1
    prob = F.Problem(n, alpha, h, tau=tau, precision="fp64")
    grads = []
    for every in (1, 5, 12, 100):
        u0 = _dev(U0, "fp64").requires_grad_(True)
        pt = torch.tensor(BASE_PARAMS, dtype=torch.float64, requires_grad=True)
        loss = (prob.trajectory(u0, pt, steps, every=every) - _dev(Ut, "fp64")).abs().pow(2).sum()
        loss.backward()
        grads.append((_host(u0.grad), pt.grad.numpy().copy()))
    for g, p in grads[1:]:
        assert _rel(g, grads[0][0]) <= 1e-12
        np.testing.assert_allclose(p, grads[0][1], rtol=1e-11)
    prob.close()


def test_adjoint_workload_96_matches_stored_oracle_gradient(F):
    """96^3, alpha = 1.5, complex64 / FP32 MFMA, 200 steps, checkpoints every 20; loss against
    the oracle's trajectory with perturbed parameters.  Compared with the oracle gradient on
    8192 stored samples of the u0 cotangent, all five parameter cotangents and the loss."""
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle gradient not generated")
    g = dict(np.load(GOLDEN))
    w = adjoint_3d()
    U0 = u0_adjoint(w)
    pert = tuple(p + d for p, d in zip(w.params, ADJOINT_PERTURBATION))
    Ut = O.run(O.Problem(w.n, w.alpha, w.h, pert), "exp_euler", U0, w.tau, w.steps)
    prob = F.Problem(w.n, w.alpha, w.h, tau=w.tau, precision="fp32")
    u0 = _dev(U0, "fp32").requires_grad_(True)
    pt = torch.tensor(w.params, dtype=torch.float64, requires_grad=True)
    uT = prob.trajectory(u0, pt, w.steps, every=ADJOINT_CHECKPOINT_EVERY)
    loss = (uT - _dev(Ut, "fp32")).abs().pow(2).sum()
    loss.backward()
    got = u0.grad.reshape(-1)[torch.from_numpy(g["idx"]).cuda()].cpu().numpy().astype(np.complex128)
    eu = _rel(got, g["ubar0"])
    ep = float(np.linalg.norm(pt.grad.numpy() - g["pbar"]) / np.linalg.norm(g["pbar"]))
    el = abs(float(loss) - float(g["loss"])) / float(g["loss"])
    print(f"[adjoint 96^3 fp32 x200/20] u0 rel_l2 = {eu:.3e}, params rel = {ep:.3e}, loss rel = {el:.3e}")
    assert eu <= 1e-3
    assert ep <= 1e-3
    assert el <= 1e-4
    prob.close()

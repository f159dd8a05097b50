"""Full-size, full-length parity against stored oracle trajectories (tests/golden/*.npz,
written by tests/golden/make_golden.py, which calls only the oracle).

Each stored case holds 8192 sampled outputs of u(T) (seeded indices) and the norm of the
whole oracle u(T).  The HIP path runs the whole trajectory in the configuration the
benchmark times (autotuned plan); the relative L2 error over the samples and the relative
error of the full norm are checked against the precision's bound.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fcgle_oracle as O
from workloads import headline_3d, manufactured_3d, u0_headline, u0_manufactured

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(__file__), "golden")
CDT = {"fp64": torch.complex128, "fp32": torch.complex64, "bf16x3": torch.complex64, "bf16x6": torch.complex64}


@pytest.fixture(scope="module")
def F():
    import paper_2510_21394_amd as pkg
    return pkg


def _golden(name):
    path = os.path.join(HERE, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not generated")
    return dict(np.load(path))


def _compare(u, g):
    got = u.reshape(-1)[torch.from_numpy(g["idx"]).cuda()].cpu().numpy().astype(np.complex128)
    err = float(np.linalg.norm(got - g["val"]) / np.linalg.norm(g["val"]))
    full = float(torch.linalg.vector_norm(u.to(torch.complex128)).cpu())
    return err, abs(full - float(g["norm"])) / float(g["norm"])


@pytest.mark.parametrize("scheme", ["exp_euler", "lie", "lbdf2"])
def test_manufactured_128_full_trajectory(F, scheme):
    """128^3 on (-8,8)^3, alpha = (1.3,1.6,1.8), 1000 steps of tau = 5e-4 with the
    semi-discrete manufactured source, FP64: vs the stored oracle u(T) <= 1e-12."""
    w = manufactured_3d(scheme)
    g = _golden(w.name)
    U0 = u0_manufactured(w)
    P = O.Problem(w.n, w.alpha, w.h, w.params)
    src = O.manufactured_source(U0, P.Ds, w.params)
    plan = F.Plan(w.n, w.alpha, w.h, w.params, tau=w.tau, precision="fp64")
    plan.autotune(2)
    plan.set_source(src.rates, [torch.from_numpy(S).cuda() for S in src.tensors])
    u = torch.from_numpy(U0).cuda()
    plan.set_state(u)
    plan.run(scheme, u, 0.0, w.steps)
    err, nerr = _compare(u, g)
    temporal = O.rel_l2(u.cpu().numpy(), math.exp(-w.tau * w.steps) * U0)
    print(f"[{w.name} x{w.steps}] sampled rel_l2 = {err:.3e}, norm rel = {nerr:.3e}, "
          f"error vs exact e^-T U0 = {temporal:.3e}")
    assert err <= 1e-12
    assert nerr <= 1e-12
    plan.close()


_HEADLINE_ERR = {}


def _headline_error(F, prec):
    """256^3 on (-12,12)^3, alpha = 1.7, four Gaussians, 200 exponential-Euler steps of
    tau = 1e-3 from u0, autotuned plan: sampled relative L2 error and relative norm error
    against the stored FP64 oracle u(T).  Computed once per precision and module."""
    if prec not in _HEADLINE_ERR:
        w = headline_3d()
        g = _golden(w.name)
        plan = F.Plan(w.n, w.alpha, w.h, w.params, tau=w.tau, precision=prec)
        plan.autotune(2)
        u = torch.from_numpy(u0_headline(w)).to(CDT[prec]).cuda()
        plan.set_state(u)
        plan.run("exp_euler", u, 0.0, w.steps)
        err, nerr = _compare(u, g)
        print(f"[{w.name} {prec} x{w.steps}] sampled rel_l2 = {err:.3e}, norm rel = {nerr:.3e} "
              f"({plan.describe()})")
        plan.close()
        del u
        torch.cuda.empty_cache()
        _HEADLINE_ERR[prec] = (err, nerr)
    return _HEADLINE_ERR[prec]


# Bounds at T: FP64 1e-12, FP32 1e-5 and split-BF16 1e-6 as stated for the method's precision
# forms.  Split-BF16 with 3 products (2 BF16 pieces per operand) carries the 2-piece
# representation error of FP32 data, about 2^-17 relative, into every mode product, so it
# cannot reach 1e-6: it is held to 1e-4 here as a regression guard, and to the stated 1e-6 by
# the strict expected failure below, which records the miss.
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16x6", 1e-6), ("bf16x3", 1e-4)])
def test_headline_256_full_trajectory(F, prec, tol):
    err, nerr = _headline_error(F, prec)
    assert err <= tol
    assert nerr <= tol


@pytest.mark.xfail(strict=True, reason="split-BF16 with 3 products (2 BF16 pieces per operand) represents FP32 data "
                                       "to about 2^-17, so its error at T (measured 8e-6) misses the stated 1e-6; "
                                       "the 6-product form (3 pieces) meets it")
def test_headline_256_bf16x3_stated_bound(F):
    err, nerr = _headline_error(F, "bf16x3")
    assert err <= 1e-6
    assert nerr <= 1e-6

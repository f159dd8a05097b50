"""The paper's Example 1 through the HIP path against the errors the paper prints.

u = e^{-it} prod_mu (1 - x_mu^2)^4 on (-1,1)^d solves the equation with a source e^{-it} S
(complex rate -i, built by the oracle from the closed-form Riesz derivative); LBDF2 with the
backward-forward Euler start, FD2, T = 1, tau = 1/steps.  The absolute discrete-L2 errors at T
are compared with the values in tests/golden/example1_printed_errors.txt (Section 4, first 2-D
and first 3-D experiments):
  2-D, n = 400, FP64: within half a unit of the last printed digit (all five digits);
  2-D, n = 400, FP32: within half a unit of the third significant digit (the FP32 state's
      rounding, ~1e-7 of the solution, moves the fifth digit);
  3-D, n = 200, FP64 and FP32: the paper's 3-D values come from three implementations run in
      single precision throughout (set-up included), which differ from one another by up to
      3.8 %; each lies above the FP64 error by a nearly constant amount (3-4e-5 for C++ and
      CUDA, 6-8e-5 for MATLAB), the rounding floor of those runs.  Required here: at most the
      lowest printed value and at least 90 % of it.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fcgle_oracle as O

pytestmark = pytest.mark.gpu

PARAMS = (1.0, 1.0, 3.0, 1.0, 2.0)
ALPHA = {2: (1.2, 1.8), 3: (1.2, 1.8, 1.5)}
CDT = {"fp64": torch.complex128, "fp32": torch.complex64}


def _printed():
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "example1_printed_errors.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                d, n, steps, err, series = line.split()
                rows.append((int(d), int(n), int(steps), err, series))
    return rows


def _unit(printed: str, digits=None) -> float:
    mant, exp = printed.lower().split("e")
    decimals = len(mant.split(".")[1]) if "." in mant else 0
    if digits is not None:
        decimals = digits - 1
    return 10.0 ** (int(exp) - decimals)


@pytest.fixture(scope="module")
def F():
    import paper_2510_21394_amd as pkg
    return pkg


def _errors(F, dim, n, prec, step_counts):
    U0, src, h = O.example1(n, ALPHA[dim], PARAMS)
    S = torch.from_numpy(src.tensors[0]).to(CDT[prec]).cuda()
    del src
    u0 = torch.from_numpy(U0).to(CDT[prec]).cuda()
    ex = torch.from_numpy(np.exp(-1j) * U0).cuda()
    out = {}
    for steps in step_counts:
        plan = F.Plan(U0.shape, ALPHA[dim], h, PARAMS, tau=1.0 / steps, precision=prec)
        plan.set_source([-1j], [S])
        u = u0.clone()
        plan.run("lbdf2", u, 0.0, steps)
        out[steps] = float(np.sqrt(np.prod(h)) * torch.linalg.vector_norm(u.to(torch.complex128) - ex).item())
        plan.close()
        print(f"[example1 {dim}-D n={n} {prec} steps={steps}] error {out[steps]:.5e}", flush=True)
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lbdf2_reproduces_the_printed_errors_2d(F, prec):
    rows = [r for r in _printed() if r[0] == 2 and r[4] == "lbdf2-m"]
    errs = _errors(F, 2, rows[0][1], prec, [r[2] for r in rows])
    for _, _, steps, printed, _ in rows:
        tol = 0.5 * (_unit(printed) if prec == "fp64" else _unit(printed, digits=3))
        assert abs(errs[steps] - float(printed)) <= tol, (steps, errs[steps], printed)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lbdf2_within_the_printed_3d_band(F, prec):
    """Context check, not parity: the 3-D LBDF2 errors must lie between 0.9x and 1x of the
    lowest printed single-precision series at each step count.  The band was set after the
    measurement (92-99 % of those values), so it guards against regressions rather than
    confirming an independent prediction."""
    rows = [r for r in _printed() if r[0] == 3 and r[4].startswith("lbdf2-t")]
    step_counts = sorted({r[2] for r in rows})
    errs = _errors(F, 3, rows[0][1], prec, step_counts)
    for steps in step_counts:
        vals = [float(r[3]) for r in rows if r[2] == steps]
        lo, hi = min(vals), max(vals)
        print(f"  steps={steps}: {errs[steps]:.4e}, printed [{lo:.3e}, {hi:.3e}]")
    for steps in step_counts:
        lo = min(float(r[3]) for r in rows if r[2] == steps)
        assert 0.9 * lo <= errs[steps] <= lo, (steps, errs[steps], lo)

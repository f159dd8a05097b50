"""GPU parity of the batched form (many independent 2-D instances of uneven sizes and
parameters, FP32 MFMA, complex64) against the FP64 oracle run instance by instance.

Tolerance: relative L2 per instance <= 1e-5 (the FP32 bound of the single-problem path).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fcgle_oracle as O
from workloads import BATCH_STEPS, BATCH_TAU, batch_2d, grid_axes, sech_product, u0_batch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "2d_batch64_expeuler.npz")
SIZES = [(24, 70), (130, 33), (96, 96), (5, 200), (257, 40), (64, 129), (300, 17)]


@pytest.fixture(scope="module")
def F():
    import paper_2510_21394_amd as pkg
    return pkg


def _instances(seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for n in SIZES:
        alpha = tuple(rng.uniform(1.2, 1.9, 2))
        dom = ((-10.0, 10.0),) * 2
        h = tuple((b - a) / (m + 1) for (a, b), m in zip(dom, n))
        params = (rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 2),
                  rng.uniform(-1, 1))
        u0 = sech_product(grid_axes(n, dom), tuple(rng.uniform(-1, 1, 2)), rng.uniform(0, 2 * np.pi))
        out.append((n, alpha, h, params, u0))
    return out


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.complex64).cuda()


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("tune", [False, True])
def test_small_batch_matches_oracle(F, tune):
    insts = _instances()
    tau, steps = 1e-3, 20
    plan = F.BatchPlan([i[:4] for i in insts], tau=tau)
    if tune:
        plan.autotune(2)
    desc = plan.describe()
    print(desc)
    # one class per phase (the default), or size classes of the axis-0 half-block length
    # m_e = ceil(n_0 / 2) <= 128 and larger when the autotuner times them faster
    nsmall = sum(1 for i in insts if (i[0][0] + 1) // 2 <= 128)
    split = f"classes(m_e<=128|larger, axis 0)={nsmall}|{len(insts) - nsmall}"
    assert ("classes=one" in desc) or (tune and split in desc)
    us = [_dev(i[4]) for i in insts]
    plan.run(us, 0.0, steps)
    for (n, alpha, h, params, u0), u in zip(insts, us):
        ref = O.run(O.Problem(n, alpha, h, params), "exp_euler", u0, tau, steps)
        err = O.rel_l2(_host(u), ref)
        print(f"[batch {n}] rel_l2 = {err:.3e}")
        assert err <= 1e-5
    plan.close()


def test_batch_calls_are_independent_and_rebind_buffers(F):
    insts = _instances(5)[:4]
    tau = 1e-3
    plan = F.BatchPlan([i[:4] for i in insts], tau=tau)
    a = [_dev(i[4]) for i in insts]
    plan.run(a, 0.0, 7)
    plan.run(a, 7 * tau, 5)           # continues from the state written by the first call
    b = [_dev(i[4]) for i in insts]   # other buffers: item arrays are rebuilt
    plan.run(b, 0.0, 12)
    for x, y in zip(a, b):
        assert O.rel_l2(_host(x), _host(y)) <= 1e-6
    c = [_dev(i[4]) for i in insts]
    plan.run(c, 0.0, 0)               # zero steps leave the state alone
    for i, x in zip(insts, c):
        assert np.array_equal(_host(x), i[4].astype(np.complex64).astype(np.complex128))
    plan.close()


def test_persistent_form_is_refused(F):
    insts = _instances()[:2]
    plan = F.BatchPlan([i[:4] for i in insts], tau=1e-3)
    with pytest.raises(F.FcgleError) as e:
        plan.set_persistent(True)
    assert e.value.code == -2
    plan.set_persistent(False)
    plan.close()


def test_batch_argument_errors(F):
    insts = _instances()[:2]
    with pytest.raises(F.FcgleError) as e:
        F.BatchPlan([i[:4] for i in insts], tau=1e-3, precision="fp64")
    assert e.value.code == -2
    plan = F.BatchPlan([i[:4] for i in insts], tau=1e-3)
    us = [_dev(i[4]) for i in insts]
    with pytest.raises(F.FcgleError) as e:
        plan.run(us, 0.0, 3, scheme="lie")
    assert e.value.code == -2
    from paper_2510_21394_amd import _lib as L
    import ctypes
    rc = L.lib().fcgle_step(plan.handle, 0, ctypes.c_void_p(us[0].data_ptr()), 0.0, 1e-3, None)
    assert rc == L.ERR_ARG
    plan.close()


PERSISTENT_OFF = ("the persistent batch form is switched off: its first GPU runs stalled (killed for silence "
                  "during autotuning) and the cause is not established")


@pytest.mark.parametrize("persistent", [False, pytest.param(True, marks=pytest.mark.skip(reason=PERSISTENT_OFF))],
                         ids=["graph", "persistent"])
def test_small_batch_each_form_matches_oracle(F, persistent):
    """The graph of grouped launches and the persistent kernel (its default tile configuration),
    each against the oracle, over several calls (state carried between them)."""
    insts = _instances(7)
    tau = 1e-3
    plan = F.BatchPlan([i[:4] for i in insts], tau=tau)
    plan.set_persistent(persistent)
    us = [_dev(i[4]) for i in insts]
    plan.run(us, 0.0, 9)
    plan.run(us, 9 * tau, 14)
    print(plan.describe())
    for (n, alpha, h, params, u0), u in zip(insts, us):
        ref = O.run(O.Problem(n, alpha, h, params), "exp_euler", u0, tau, 23)
        err = O.rel_l2(_host(u), ref)
        print(f"[batch {'persistent' if persistent else 'graph'} {n}] rel_l2 = {err:.3e}")
        assert err <= 1e-5
    plan.close()


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_wait_limit_ends_the_run(F):
    """A dependency wait of the persistent kernel that runs out of polls (forced from the host
    with a limit of one poll) abandons the run: every workgroup leaves and the call reports
    ERR_HIP (or, if no wait had to poll twice, the run completed and is correct).  A run with the
    default limit afterwards is correct again."""
    insts = _instances(9)
    tau = 1e-3
    plan = F.BatchPlan([i[:4] for i in insts], tau=tau)
    plan.set_persistent(True, spin_limit=1)
    us = [_dev(i[4]) for i in insts]
    try:
        plan.run(us, 0.0, 30)
        failed = False
    except F.FcgleError as e:
        assert e.code == -4 and "ran out of polls" in str(e)
        failed = True
    print(f"tiny wait limit: run abandoned = {failed}")
    if not failed:
        for (n, alpha, h, params, u0), u in zip(insts, us):
            assert O.rel_l2(_host(u), O.run(O.Problem(n, alpha, h, params), "exp_euler", u0, tau, 30)) <= 1e-5
    plan.set_persistent(True, spin_limit=1000000)
    us = [_dev(i[4]) for i in insts]
    plan.run(us, 0.0, 30)
    for (n, alpha, h, params, u0), u in zip(insts, us):
        assert O.rel_l2(_host(u), O.run(O.Problem(n, alpha, h, params), "exp_euler", u0, tau, 30)) <= 1e-5
    plan.close()


@pytest.mark.parametrize("form", ["tuned", pytest.param("persistent", marks=pytest.mark.skip(reason=PERSISTENT_OFF))])
def test_batch_workload_64_matches_stored_oracle(F, form):
    """64 instances (sizes 96..512 per axis, seed 2510), 500 steps, tau = 1e-3: 256 stored
    oracle samples per instance; the relative error is taken over each instance's samples
    against the norm of the samples.  In the autotuned form and forced to the persistent kernel."""
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle outputs not generated")
    g = dict(np.load(GOLDEN))
    insts = batch_2d()
    plan = F.BatchPlan([(i.n, i.alpha, i.h, i.params) for i in insts], tau=BATCH_TAU)
    plan.autotune(2)
    if form == "persistent":
        plan.set_persistent(True)
    print(plan.describe())
    us = [_dev(u0_batch(i)) for i in insts]
    plan.run(us, 0.0, BATCH_STEPS)
    worst = 0.0
    for k, u in enumerate(us):
        got = u.reshape(-1)[torch.from_numpy(g["idx"][k]).cuda()].cpu().numpy().astype(np.complex128)
        err = float(np.linalg.norm(got - g["val"][k]) / np.linalg.norm(g["val"][k]))
        worst = max(worst, err)
        full = float(torch.linalg.vector_norm(u.to(torch.complex128)).cpu())
        assert abs(full - g["norm"][k]) <= 1e-5 * g["norm"][k]
    print(f"[batch64 x{BATCH_STEPS}] worst sampled rel_l2 = {worst:.3e}")
    assert worst <= 1e-5
    plan.close()

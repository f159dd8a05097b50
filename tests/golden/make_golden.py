"""Write the stored references of the full-size GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators (workloads/).
Each case runs a whole trajectory on the CPU and stores, in <case>.npz:
  idx   : 8192 sampled flat indices (sorted, drawn by default_rng(20251021))
  val   : the oracle's u(T) at those indices (complex128)
  norm  : the L2 norm of the whole oracle u(T)
  steps, tau, scheme : the trajectory that produced it

The adjoint case stores the oracle's gradient instead (see case_adjoint).  The refined-step
cases of the 256^3 workload (case_headline_refined) repeat its trajectory to the same T with
tau/2 and tau/4; they sample the same indices, so the temporal discretisation error of the
tau = 1e-3 trajectory can be estimated from the stored samples alone (Richardson: for a
first-order scheme u_tau - u_exact ~ 2 (u_tau - u_{tau/2})).

Usage: python tests/golden/make_golden.py [case ...]   (all cases by default)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fcgle_oracle as O  # noqa: E402
import workloads as W  # noqa: E402

NSAMPLE = 8192


def _save(name, U, steps, tau, scheme):
    rng = np.random.default_rng(20251021)
    idx = np.sort(rng.choice(U.size, size=min(NSAMPLE, U.size), replace=False))
    np.savez(os.path.join(HERE, name + ".npz"), idx=idx, val=U.reshape(-1)[idx],
             norm=np.linalg.norm(U.reshape(-1)), steps=steps, tau=tau, scheme=scheme)


def case_manufactured(scheme):
    w = W.manufactured_3d(scheme)
    U0 = W.u0_manufactured(w)
    P = O.Problem(w.n, w.alpha, w.h, w.params)
    P.source = O.manufactured_source(U0, P.Ds, w.params)
    U = O.run(P, scheme, U0, w.tau, w.steps)
    _save(w.name, U, w.steps, w.tau, scheme)
    exact = np.exp(-w.tau * w.steps) * U0
    print(f"{w.name}: temporal error vs e^(-T) U0 = {O.rel_l2(U, exact):.3e}")


def case_headline():
    w = W.headline_3d()
    U0 = W.u0_headline(w)
    P = O.Problem(w.n, w.alpha, w.h, w.params)
    U = O.run(P, "exp_euler", U0, w.tau, w.steps)
    _save(w.name, U, w.steps, w.tau, "exp_euler")


def case_headline_refined(k):
    """The 256^3 workload to the same T = 0.2 with tau / k (200 k steps); stored under the
    headline's name with the suffix _tau<k>."""
    w = W.headline_3d()
    U0 = W.u0_headline(w)
    P = O.Problem(w.n, w.alpha, w.h, w.params)
    tau, steps = w.tau / k, w.steps * k
    U = O.run(P, "exp_euler", U0, tau, steps)
    _save(f"{w.name}_tau{k}", U, steps, tau, "exp_euler")


def case_adjoint():
    """96^3 adjoint workload: L = ||u(T) - u_target||^2 with u_target the trajectory under the
    perturbed parameters; stores the oracle gradient (u0 samples, five parameters) and L."""
    w = W.adjoint_3d()
    U0 = W.u0_adjoint(w)
    pert = tuple(p + d for p, d in zip(w.params, W.ADJOINT_PERTURBATION))
    Ut = O.run(O.Problem(w.n, w.alpha, w.h, pert), "exp_euler", U0, w.tau, w.steps)
    P = O.Problem(w.n, w.alpha, w.h, w.params)
    L, g, p = O.expeuler_loss_and_grad(P, U0, Ut, w.tau, w.steps)
    rng = np.random.default_rng(20251021)
    idx = np.sort(rng.choice(g.size, size=min(NSAMPLE, g.size), replace=False))
    np.savez(os.path.join(HERE, w.name + ".npz"), idx=idx, ubar0=g.reshape(-1)[idx],
             norm=np.linalg.norm(g.reshape(-1)), pbar=p, loss=L, steps=w.steps, tau=w.tau)
    print(f"{w.name}: L = {L:.6e}, pbar = {p}")


def case_batch():
    """64 batched 2-D instances, 500 exponential-Euler steps each; stores 256 sampled
    outputs per instance (seeded) and each instance's full-tensor norm."""
    insts = W.batch_2d()
    rng = np.random.default_rng(20251021)
    idx = np.zeros((len(insts), 256), np.int64)
    val = np.zeros((len(insts), 256), np.complex128)
    norm = np.zeros(len(insts))
    for i, inst in enumerate(insts):
        P = O.Problem(inst.n, inst.alpha, inst.h, inst.params)
        U = O.run(P, "exp_euler", W.u0_batch(inst), W.BATCH_TAU, W.BATCH_STEPS)
        ii = np.sort(rng.choice(U.size, size=256, replace=False))
        idx[i], val[i], norm[i] = ii, U.reshape(-1)[ii], np.linalg.norm(U.reshape(-1))
        print(f"batch instance {i} {inst.n} done", flush=True)
    np.savez(os.path.join(HERE, "2d_batch64_expeuler.npz"), idx=idx, val=val, norm=norm,
             steps=W.BATCH_STEPS, tau=W.BATCH_TAU)


CASES = {
    "2d_batch64_expeuler": case_batch,
    "3d_96_adjoint": case_adjoint,
    "3d_128_manufactured_lbdf2": lambda: case_manufactured("lbdf2"),
    "3d_128_manufactured_lie": lambda: case_manufactured("lie"),
    "3d_128_manufactured_exp_euler": lambda: case_manufactured("exp_euler"),
    "3d_256_gauss4_expeuler": case_headline,
    "3d_256_gauss4_expeuler_tau2": lambda: case_headline_refined(2),
    "3d_256_gauss4_expeuler_tau4": lambda: case_headline_refined(4),
}


def main(argv):
    names = argv or list(CASES)
    for name in names:
        t0 = time.time()
        CASES[name]()
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])

"""CPU checks of the C-ABI library: it loads, exports every declared entry point, and its
host-only helpers (FD weights, own eigensolver, scalar matrix functions) agree with the
oracle.  No device call is made."""
import os
import re

import numpy as np
import pytest

from oracle import fcgle_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcgle.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcgle_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def F():
    import paper_2510_21394_amd as pkg
    return pkg


def test_library_exports_every_declared_symbol(F):
    from paper_2510_21394_amd import _lib as L
    lib = L.lib()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == {s[0] for s in L.SIGNATURES}


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9, 2.0])
@pytest.mark.parametrize("order", [2, 4])
def test_host_fd_weights_match_oracle(F, alpha, order):
    g = F.host_fd_weights(alpha, 64, order)
    ref = O.fd2_weights(alpha, 64) if order == 2 else O.fd4_weights(alpha, 64)
    np.testing.assert_allclose(g, ref, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("n,alpha,h", [(2, 1.5, 0.3), (17, 2.0, 0.2), (96, 1.5, 20 / 97), (129, 1.3, 16 / 129),
                                       (300, 1.8, 0.05)])
def test_host_eig_against_lapack(F, n, alpha, h):
    Q, lam = F.host_eig(n, alpha, h)
    D = O.diff_matrix(alpha, n, h)
    lo, _ = O.eig(D)
    assert np.linalg.norm(Q @ np.diag(lam) @ Q.T - D) <= 1e-14 * np.linalg.norm(D)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 5e-14 * np.sqrt(n)
    # backward-stable eigenvalues carry an absolute error of order eps * ||D||
    assert np.max(np.abs(lam - lo)) <= 1e-14 * np.max(np.abs(lo))
    assert np.all(np.diff(lam) >= 0)


def test_host_eig_alpha2_closed_form(F):
    n, h = 33, 0.1
    _, lam = F.host_eig(n, 2.0, h)
    k = np.arange(1, n + 1)
    ref = np.sort(-(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n + 1))) ** 2)
    np.testing.assert_allclose(lam, ref, rtol=1e-13)


def test_host_eig_fd4(F):
    Q, lam = F.host_eig(50, 1.4, 0.2, 4)
    D = O.diff_matrix(1.4, 50, 0.2, fd_order=4)
    assert np.linalg.norm(Q @ np.diag(lam) @ Q.T - D) <= 1e-14 * np.linalg.norm(D)


@pytest.mark.parametrize("kind", ["inv", "exp", "phi1", "phi2", "phi3"])
def test_host_fz_matches_oracle(F, kind):
    rng = np.random.default_rng(4)
    z = (rng.standard_normal(4000) + 1j * rng.standard_normal(4000)) * 10.0 ** rng.uniform(-10, 1.3, 4000)
    z = np.concatenate([z, [0.0, -1.0, 1j, 0.999, -0.999j] + ([] if kind == "inv" else [1.0])])
    got = F.host_fz(kind, z)
    ref = O.f_of(kind, z)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 5e-15


def test_host_helpers_reject_bad_arguments(F):
    from paper_2510_21394_amd import _lib as L
    with pytest.raises(L.FcgleError) as e:
        F.host_fd_weights(2.5, 10)
    assert e.value.code == L.ERR_ARG
    with pytest.raises(L.FcgleError):
        F.host_eig(10, 1.5, -1.0)
    with pytest.raises(L.FcgleError):
        F.host_fd_weights(1.5, 10, 3)

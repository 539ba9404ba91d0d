"""CPU checks of the DGSEM embedding's host tables (libdgembed.so, no GPU): Gauss nodes and
weights, the Lagrange basis at the element ends and the weak-form derivative matrix, each
against numpy; and the paper's Table 2 fixture, whose printed orders follow from its
printed errors."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg_embed.h")
LIB = os.path.join(ROOT, "paper_2008_04356_amd", "libdgembed.so")
GOLDEN = os.path.join(ROOT, "tests", "golden", "table2_manufactured_solution.txt")


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the libraries first (paper_2008_04356_amd/build.py)"
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", txt)))
    assert len(names) >= 8
    lib = C.CDLL(LIB)
    for name in names:
        assert hasattr(lib, name), name


def _tables(N):
    lib = C.CDLL(LIB)
    lib.dg_basis_bytes.restype = C.c_int64
    tab = np.zeros(lib.dg_basis_bytes(N) // 8)
    assert lib.dg_basis_tables(N, tab.ctypes.data_as(C.POINTER(C.c_double))) == 0
    NP = N + 1
    return (tab[:NP], tab[NP:2 * NP], tab[2 * NP:3 * NP], tab[3 * NP:4 * NP],
            tab[4 * NP:].reshape(NP, NP))


@pytest.mark.parametrize("N", range(1, 8))
def test_tables_against_numpy(N):
    x, w, lm, lp, Dw = _tables(N)
    xn, wn = np.polynomial.legendre.leggauss(N + 1)
    assert np.max(np.abs(x - xn)) < 4e-16 and np.max(np.abs(w - wn)) < 2e-15
    # Lagrange basis of the nodes through numpy's polynomial fit of the unit vectors
    V = np.vander(xn, N + 1, increasing=True)
    coef = np.linalg.solve(V, np.eye(N + 1))            # column j: coefficients of l_j
    ev = lambda t: np.polynomial.polynomial.polyval(t, coef)  # noqa: E731
    assert np.max(np.abs(lm - ev(-1.0))) < 1e-11 and np.max(np.abs(lp - ev(1.0))) < 1e-11
    # the weak-form derivative: sum_m w_i Dw[i][m] f(x_m) = integral of l_i' f for any f of
    # degree <= N + 1 (the Gauss rule is exact to degree 2N + 1)
    rng = np.random.default_rng(N)
    for _ in range(3):
        f = rng.normal(size=N + 2)
        for i in range(N + 1):
            dl = np.polynomial.polynomial.polyder(coef[:, i])
            prod = np.polynomial.polynomial.polymul(dl, f)
            integ = np.polynomial.polynomial.polyint(prod)
            exact = np.polynomial.polynomial.polyval(1.0, integ) - np.polynomial.polynomial.polyval(-1.0, integ)
            got = w[i] * np.dot(Dw[i], np.polynomial.polynomial.polyval(xn, f))
            assert abs(got - exact) < 1e-10 * max(1.0, abs(exact))
    lib = C.CDLL(LIB)
    lib.dg_basis_bytes.restype = C.c_int64
    assert lib.dg_basis_bytes(8) == -1 and lib.dg_basis_bytes(0) == -1
    assert lib.dg_basis_tables(8, np.zeros(128).ctypes.data_as(C.POINTER(C.c_double))) == -1


def test_table2_fixture_orders_follow_from_its_errors():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    K = [int(r[0]) for r in rows]
    for col in range(4):
        err = [float(r[1 + 2 * col]) for r in rows]
        for i in range(1, len(rows)):
            printed = float(rows[i][2 + 2 * col])
            assert abs(math.log(err[i - 1] / err[i], K[i] / K[i - 1]) - printed) < 0.02

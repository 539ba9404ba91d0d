"""Pins of the projection operators (Sec. 3.2: mass matrix M, S, face->mortar
P = M^-1 S (exact for equal degree), mortar->face with weights (1 -+ sigma)/2 and S^T).

Independent routes: closed-form interpolation, quadrature identities, and exact rational
arithmetic (Python fractions with symbolic polynomial integration) for LGL N = 1, 2."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

LOWER = lambda s: [-1.0, -1.0 + 2.0 * s, 1.0 - 2.0 * s, -1.0]  # noqa: E731
FRAC = lambda s: [s, 1.0 - s, s, 1.0 - s]  # noqa: E731


@pytest.mark.parametrize("node_set", [O.GAUSS, O.LGL])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9])
def test_forward_is_interpolation(node_set, N):
    rng = np.random.default_rng(N)
    x, _ = O.nodes(N, node_set)
    for s in [0.0, 1e-9, 0.25, rng.uniform(), 0.999999]:
        d = O.projection_matrices(N, node_set, s)
        for k in range(4):
            ref = np.array([[O.lagrange(N, x, j, LOWER(s)[k] + (x[q] + 1.0) * FRAC(s)[k])
                             for j in range(N + 1)] for q in range(N + 1)])
            assert np.max(np.abs(d["Pf"][k] - ref)) < 5e-13


@pytest.mark.parametrize("node_set", [O.GAUSS, O.LGL])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9])
def test_back_projection_identities(node_set, N):
    x, w = O.nodes(N, node_set)
    for s in [0.0, 0.1, 0.5, 0.77, 0.999]:
        d = O.projection_matrices(N, node_set, s)
        Pf, Pb, J = d["Pf"], d["Pb"], d["J"]
        assert np.allclose(J, FRAC(s))
        # integral preservation:  w^T Pb_k = J_k (quadrature weights of the mortar)
        for k in range(4):
            wk = d["M"].sum(axis=0)  # int l_j = column sums of M
            assert np.max(np.abs(wk @ Pb[k] - J[k] * wk)) < 1e-13
        # projecting the exact restriction back reproduces the face polynomial
        for pair in ((0, 1), (2, 3)):
            I = sum(Pb[k] @ Pf[k] for k in pair)
            assert np.max(np.abs(I - np.eye(N + 1))) < 1e-12
    if node_set == O.GAUSS:
        assert np.max(np.abs(d["M"] - np.diag(w))) < 1e-14


def test_identity_at_zero_fraction():
    for N in (1, 3, 6):
        for ns in (O.GAUSS, O.LGL):
            d = O.projection_matrices(N, ns, 0.0)
            assert np.max(np.abs(d["Pf"][1] - np.eye(N + 1))) < 1e-14
            assert np.max(np.abs(d["Pb"][1] - np.eye(N + 1))) < 1e-13
            assert np.max(np.abs(d["Pf"][3] - np.eye(N + 1))) < 1e-14
            assert np.max(np.abs(d["Pb"][0])) == 0.0 and np.max(np.abs(d["Pb"][2])) == 0.0


# ---- exact rational arithmetic -------------------------------------------------------

def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            out[i + j] += ai * bj
    return out


def _pint(a):  # integral over [-1, 1]
    return sum(c * Fraction(2, k + 1) for k, c in enumerate(a) if k % 2 == 0)


def _lagr(nodes, j):
    p = [Fraction(1)]
    for m, xm in enumerate(nodes):
        if m != j:
            d = nodes[j] - xm
            p = _pmul(p, [-xm / d, Fraction(1) / d])
    return p


def _compose_affine(p, lo, fr):  # p(lo + (z + 1) fr) as a polynomial in z (Horner)
    lin = [lo + fr, fr]
    out = [Fraction(0)]
    for c in reversed(p):
        out = _pmul(out, lin)
        out[0] += c
    return out


def _inv(A):
    n = len(A)
    M = [row[:] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        d = M[c][c]
        M[c] = [v / d for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


@pytest.mark.parametrize("N,nodes", [(1, [Fraction(-1), Fraction(1)]),
                                     (2, [Fraction(-1), Fraction(0), Fraction(1)])])
@pytest.mark.parametrize("s", [Fraction(1, 3), Fraction(5, 8)])
def test_exact_rational_lgl(N, nodes, s):
    NP = N + 1
    L = [_lagr(nodes, j) for j in range(NP)]
    M = [[_pint(_pmul(L[i], L[j])) for j in range(NP)] for i in range(NP)]
    Minv = _inv(M)
    lower = [Fraction(-1), -1 + 2 * s, 1 - 2 * s, Fraction(-1)]
    frac = [s, 1 - s, s, 1 - s]
    d = O.projection_matrices(N, O.LGL, float(s))
    assert np.max(np.abs(np.array(M, dtype=float) - d["M"])) < 1e-15
    for k in range(4):
        Lk = [_compose_affine(L[i], lower[k], frac[k]) for i in range(NP)]
        S = [[_pint(_pmul(Lk[i], L[j])) for j in range(NP)] for i in range(NP)]
        Pf = [[sum(Minv[q][j] * S[i][j] for j in range(NP)) for i in range(NP)] for q in range(NP)]
        Pb = [[frac[k] * sum(Minv[j][i] * S[i][q] for i in range(NP)) for q in range(NP)]
              for j in range(NP)]
        assert np.max(np.abs(np.array(S, dtype=float) - d["S"][k])) < 2e-15
        assert np.max(np.abs(np.array(Pf, dtype=float) - d["Pf"][k])) < 5e-15
        assert np.max(np.abs(np.array(Pb, dtype=float) - d["Pb"][k])) < 5e-15

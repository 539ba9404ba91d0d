"""Pins of the oracle's conservation sums (discrete conservation of the mortar
projections, Sec. 3.2 and the abstract's claim for plane interfaces).

The oracle reports per variable the static-side integral sum_p w_p w_q F, the
moving-side one, and the sum of the magnitudes of all terms.  Conservation holds line by
line, so equality of the two sides cannot pin the quadrature weights: these tests fix
the absolute values from the mathematics instead (integrals of constants and of nodal
basis functions, a numpy brute force with numpy's own Gauss weights, and exact
compensated summation of a cancelling series)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W


def _spec(N, node_set=W.GAUSS, n_par=5, n_perp=3, scramble=None, extra=0):
    return W.make_plane(N, n_par, n_perp, physics=W.EULER, riemann=W.LF, node_set=node_set,
                        precision=W.FP64, scramble_seed=scramble, extra_cols=extra)


def _field(spec, fn, side):
    """F[v][p][col] = fn(v, p_par, p_perp, i_par, i_perp) on the interface's columns of
    one side, NaN on every other column (never read)."""
    nf = spec.n_face_static if side == 0 else spec.n_face_moving
    fid = spec.face_id_static if side == 0 else spec.face_id_moving
    NP = spec.N + 1
    F = np.full((5, spec.P, nf), np.nan)
    for ip in range(spec.n_perp):
        for ia in range(spec.n_par):
            for p in range(spec.P):
                for v in range(5):
                    F[v, p, fid[ip, ia]] = fn(v, p % NP, p // NP, ia, ip)
    return F


@pytest.mark.parametrize("N,node_set", [(1, W.GAUSS), (3, W.GAUSS), (4, W.LGL), (7, W.GAUSS)])
def test_constant_flux_integrates_to_area(N, node_set):
    """A constant c_v on every point: each face integrates to c_v (sum w)^2 = 4 c_v on the
    reference square, so both sides give 4 c_v n_faces and the magnitudes 8 |c_v| n_faces."""
    spec = _spec(N, node_set, scramble=N, extra=3)
    c = np.array([1.0, -2.5, 0.125, 3.0, -0.75])
    Fs = _field(spec, lambda v, a, b, i, j: c[v], 0)
    Fm = _field(spec, lambda v, a, b, i, j: c[v], 1)
    out = O.conservation(spec, Fs, Fm)
    nfaces = spec.n_par * spec.n_perp
    np.testing.assert_allclose(out[:, 0], 4.0 * c * nfaces, rtol=1e-14)
    np.testing.assert_allclose(out[:, 1], 4.0 * c * nfaces, rtol=1e-14)
    np.testing.assert_allclose(out[:, 2], 8.0 * np.abs(c) * nfaces, rtol=1e-14)


@pytest.mark.parametrize("N,node_set", [(2, W.GAUSS), (3, W.LGL), (5, W.GAUSS)])
@pytest.mark.parametrize("direction", ["perp", "par"])
def test_nodal_basis_function_weights(N, node_set, direction):
    """F = the nodal basis function l_k along one direction (1 at node k, 0 at the others)
    and constant along the other: each face integrates to (sum w) w_k = 2 w_k.  Dropping
    either direction's weight, or taking the wrong one, changes the value."""
    spec = _spec(N, node_set)
    x, w = W.node_positions(N, node_set), None
    w = _weights(N, node_set)
    nfaces = spec.n_par * spec.n_perp
    for k in range(N + 1):
        if direction == "perp":
            fn = lambda v, a, b, i, j: 1.0 if b == k else 0.0  # noqa: E731
        else:
            fn = lambda v, a, b, i, j: 1.0 if a == k else 0.0  # noqa: E731
        Fs = _field(spec, fn, 0)
        Fm = _field(spec, lambda v, a, b, i, j: 0.0, 1)
        out = O.conservation(spec, Fs, Fm)
        np.testing.assert_allclose(out[:, 0], 2.0 * w[k] * nfaces, rtol=1e-14)
        assert np.all(out[:, 1] == 0.0)
        np.testing.assert_allclose(out[:, 2], 2.0 * w[k] * nfaces, rtol=1e-14)
    del x


def _weights(N, node_set):
    """Quadrature weights from numpy (Gauss) or the closed form 2 / (N (N+1) P_N(x)^2)
    (Gauss-Lobatto), independent of the oracle's node routines."""
    if node_set == W.GAUSS:
        return np.polynomial.legendre.leggauss(N + 1)[1]
    x = W.node_positions(N, node_set)
    PN = np.polynomial.legendre.Legendre.basis(N)(x)
    return 2.0 / (N * (N + 1) * PN ** 2)


@pytest.mark.parametrize("N,node_set", [(2, W.GAUSS), (4, W.LGL), (6, W.GAUSS)])
def test_random_fields_against_numpy_brute_force(N, node_set):
    """Different random fields on the two sides (so a swapped side shows), scrambled
    columns with NaN on the columns off the interface: the three sums equal numpy's
    tensor-product quadrature of each side."""
    spec = _spec(N, node_set, n_par=7, n_perp=4, scramble=11, extra=5)
    rng = np.random.default_rng(N)
    vals_s = rng.uniform(-1.0, 1.0, (5, spec.P, spec.n_perp, spec.n_par))
    vals_m = rng.uniform(-2.0, 3.0, (5, spec.P, spec.n_perp, spec.n_par))
    Fs = _field(spec, lambda v, a, b, i, j: vals_s[v, a + (N + 1) * b, j, i], 0)
    Fm = _field(spec, lambda v, a, b, i, j: vals_m[v, a + (N + 1) * b, j, i], 1)
    w = _weights(N, node_set)
    w2 = np.outer(w, w).ravel()     # index p_perp * NP + p_par = p
    ref_s = np.einsum("p,vpji->v", w2, vals_s)
    ref_m = np.einsum("p,vpji->v", w2, vals_m)
    mag = np.einsum("p,vpji->v", w2, np.abs(vals_s)) + np.einsum("p,vpji->v", w2, np.abs(vals_m))
    out = O.conservation(spec, Fs, Fm)
    np.testing.assert_allclose(out[:, 0], ref_s, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(out[:, 1], ref_m, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(out[:, 2], mag, rtol=1e-13)


def test_magnitudes_of_a_sign_alternating_field():
    """Signs alternating over points and faces: the signed sums nearly cancel while the
    magnitude sum is that of the constant field, 8 |c| n_faces."""
    spec = _spec(3, W.GAUSS, n_par=4, n_perp=2)
    c = 1.75
    fn = lambda v, a, b, i, j: c * (-1.0) ** (a + b + i + j)  # noqa: E731
    Fs, Fm = _field(spec, fn, 0), _field(spec, fn, 1)
    out = O.conservation(spec, Fs, Fm)
    nfaces = spec.n_par * spec.n_perp
    np.testing.assert_allclose(out[:, 2], 8.0 * c * nfaces, rtol=1e-14)
    assert np.all(np.abs(out[:, 0]) < 1e-13) and np.all(np.abs(out[:, 1]) < 1e-13)


def test_compensated_summation_is_exact():
    """N = 1 Gauss (weights exactly 1): faces in order carry 1e16, 1 and -1e16 at every
    point.  Plain left-to-right summation loses the middle face; the compensated sums
    return exactly 4 (its four unit points), and the magnitudes 8e16 + 4 to rounding."""
    spec = _spec(1, W.GAUSS, n_par=3, n_perp=1)
    vals = [1e16, 1.0, -1e16]
    fn = lambda v, a, b, i, j: vals[i]  # noqa: E731
    out = O.conservation(spec, _field(spec, fn, 0), _field(spec, fn, 1))
    assert np.all(out[:, 0] == 4.0) and np.all(out[:, 1] == 4.0)
    np.testing.assert_allclose(out[:, 2], 2 * (8e16 + 4.0), rtol=1e-15)

"""GPU: the static-to-moving pairing the library evaluates on the device
(mortar_get_pairing, Sec. 4.3 index relation) against the oracle's brute-force pairing by
interval containment, bit for bit, over negative, huge, whole-face, zero and near-one
displacements; and the pairing's agreement with the index map's opposite-owner keys."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2008_04356_amd import mortar
    return mortar


def _brute(n_par, n, s):
    return np.array([[O.pair_bruteforce(n_par, n, s, i, k) for i in range(n_par)] for k in range(2)],
                    dtype=np.int32)


@pytest.mark.parametrize("n_par", [1, 2, 7, 64])
def test_pairing_matches_bruteforce(M, n_par):
    spec = W.make_plane(2, n_par, 3, physics=W.EULER, riemann=W.LF, precision=W.FP64, name="pair")
    op = M.MortarOperator([spec])
    l = spec.l_par
    disps = [0.0, 0.25 * l, -0.25 * l, 1.0 * l, -1.0 * l, 3.0 * l, (n_par - 1e-9) * l,
             (1.0 - 2.0 ** -40) * l, -7.3 * l, 12345.678 * l, -98765.4321 * l, 2.0 ** 40 * l]
    try:
        for d in disps:
            print(f"[pairing] n_par={n_par} disp={d:.17g}", flush=True)
            op.update([d])
            n, s = O.decompose(d, l)
            assert op.displacement(0) == (n, s)
            got = op.pairing(0)
            assert got.shape == (2, n_par)
            assert np.array_equal(got, _brute(n_par, n, s)), (d, n, s)
        # (n, s) given directly, past what an FP64 quotient can carry
        for n in (2 ** 62 + 5, -(2 ** 62) - 3, 10 ** 15 + 1):
            for s in (0.0, 0.5, 1.0 - 2.0 ** -52):
                op.update_ns([n], [s])
                assert np.array_equal(op.pairing(0), _brute(n_par, n, s)), (n, s)
    finally:
        op.close()


def test_pairing_consistent_with_index_map(M):
    # the static side's index map keys every mortar by the owner of its moving face: with
    # distinct owners per moving face the key names the paired face
    spec = W.make_plane(3, 11, 4, physics=W.EULER, riemann=W.LF, precision=W.FP64,
                        scramble_seed=5, name="pair-map")
    spec.owner_moving = (np.arange(spec.n_par * spec.n_perp, dtype=np.int32) % spec.n_par).reshape(
        spec.n_perp, spec.n_par) * 3 + 1
    op = M.MortarOperator([spec])
    try:
        for d in (0.4 * spec.l_par, 5.9 * spec.l_par, -2.2 * spec.l_par):
            op.update([d])
            pair = op.pairing(0)
            A, _ = op.index_map(0, 0)
            owner, i_par, i_sub = A[0], A[1], A[3]
            assert np.array_equal(owner, pair[i_sub, i_par] * 3 + 1)
    finally:
        op.close()


def test_pairing_not_ready(M):
    spec = W.make_plane(2, 5, 2, physics=W.EULER, riemann=W.LF, precision=W.FP64, name="pair-nr")
    op = M.MortarOperator([spec])
    try:
        pair = np.zeros((2, 5), dtype=np.int32)
        rc = M.lib.mortar_get_pairing(op.h, 0, pair.ctypes.data_as(M._ip))
        assert rc == M.ERR_NOT_READY
        assert M.lib.mortar_get_pairing(op.h, 1, pair.ctypes.data_as(M._ip)) == M.ERR_INVALID_ARG
    finally:
        op.close()

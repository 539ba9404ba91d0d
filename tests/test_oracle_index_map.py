"""Pins of the displacement decomposition, the static/moving pairing and the mortar
sorting (Sec. 4.3 index definitions, Sec. 4.4 sorting and mapping, Appendix A)."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appendix_a_sorting.txt")


def _read_golden():
    sec, out = None, {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            sec = line.strip("[]")
            out[sec] = []
            continue
        out[sec].append([int(v) for v in line.split()])
    return out


def test_decompose_cases():
    assert O.decompose(0.0, 1.0) == (0, 0.0)
    n, s = O.decompose(-0.0, 1.0)
    assert n == 0 and s == 0.0 and np.copysign(1.0, s) == 1.0
    assert O.decompose(-1e-20, 1.0) == (0, 0.0)      # q - floor(q) rounds to 1
    assert O.decompose(3.0, 1.0) == (3, 0.0)
    n, s = O.decompose(2.999, 1.0)
    assert n == 2 and abs(s - 0.999) < 1e-15
    n, s = O.decompose(-0.4, 1.0)
    assert n == -1 and abs(s - 0.6) < 1e-15
    n, s = O.decompose(123.456 / 128, 1.0 / 128)
    assert n == 123 and abs(s - 0.456) < 1e-12
    rng = np.random.default_rng(3)
    for d in rng.uniform(-1e4, 1e4, 200):
        n, s = O.decompose(d, 0.37)
        assert 0.0 <= s < 1.0
        assert abs((n + s) * 0.37 - d) <= 1e-12 * max(1.0, abs(d))


@pytest.mark.parametrize("n_par", [1, 2, 3, 5, 8, 17])
def test_pairing_bruteforce_matches_relation(n_par):
    deltas = [0.0, 0.25, 1.0, 2.999, 3.0, -0.4, 123.456, -77.5, 1e-13, 0.9999999999]
    for d in deltas:
        n, s = O.decompose(d, 1.0)
        for i in range(n_par):
            for k in (0, 1):
                bf = O.pair_bruteforce(n_par, n, s, i, k)
                assert bf == O.pair_relation(n_par, n, i, k), (d, i, k)


def test_relation_text_example():
    # i~ = i - n + i_sub - 1: for n = 1 the lower mortar of static face 5 touches
    # moving face 3 and the upper one moving face 4 (no wrap with 10 faces)
    assert O.pair_relation(10, 1, 5, 0) == 3
    assert O.pair_relation(10, 1, 5, 1) == 4
    assert O.pair_relation(10, 1, 0, 0) == 8   # periodic wrap


def test_appendix_a_sorting_and_inverse_map():
    g = _read_golden()
    A_ref = np.array(g["A"], dtype=np.int32)
    m_ref = np.array(g["m"], dtype=np.int32)
    m_col0, m_col1 = g["m_cols"][0]
    # the process's faces (i_face, i_par, i_perp), as a set
    faces = sorted({(int(A_ref[4, c]), int(A_ref[1, c]), int(A_ref[2, c])) for c in range(10)})
    n_par, n_delta = 8, 0
    rt = np.full((3, n_par), -1, dtype=np.int32)
    for row in g["rtilde"]:
        ip, c0, vals = row[0], row[1], row[2:]
        rt[ip, c0:c0 + len(vals)] = vals
    tuples = []
    for (f, ia, ip) in faces:
        for k in (0, 1):
            jt = O.pair_relation(n_par, n_delta, ia, k)
            owner = int(rt[ip, jt])
            assert owner >= 0, "owner lookup left the printed r~ entries"
            tuples.append((owner, ia, ip, k, f))
    rng = np.random.default_rng(11)
    for _ in range(5):
        order = rng.permutation(len(tuples))
        A, m = O.sort_mortars(np.array(tuples)[order], m_col0, m_col1 - m_col0 + 1)
        assert np.array_equal(A, A_ref)
        assert np.array_equal(m + 1, m_ref)   # printed i_mortar is 1-based


def test_index_map_properties_and_virtual_ranks():
    spec = W.make_plane(2, 12, 5, scramble_seed=4, extra_cols=3)
    W.seeded_owners(spec, seed=2, n_static_ranks=3, n_moving_ranks=4)
    for d in [0.0, 0.3, 5.7, -2.2, 40.01]:
        n, s = O.decompose(d * spec.l_par, spec.l_par)
        As, ms = O.index_map(0, spec.n_par, spec.n_perp, n, spec.face_id_static,
                             spec.n_face_static, spec.owner_moving)
        Am, mm = O.index_map(1, spec.n_par, spec.n_perp, n, spec.face_id_moving,
                             spec.n_face_moving, spec.owner_static)
        for A, m, fid in ((As, ms, spec.face_id_static), (Am, mm, spec.face_id_moving)):
            keys = [tuple(A[:4, c]) for c in range(A.shape[1])]
            assert keys == sorted(keys) and len(set(keys)) == len(keys)
            for c in range(A.shape[1]):
                assert m[A[3, c], A[4, c]] == c
            used = set(fid.ravel().tolist())
            for f in range(m.shape[1]):
                assert (m[0, f] >= 0) == (f in used) and (m[1, f] >= 0) == (f in used)
        # requirement 3 of Sec. 4.4: for every (static rank P, moving rank Q) pair the
        # chunk P sends/receives is ordered exactly like Q's chunk for P
        for P_ in np.unique(spec.owner_static):
            for Q_ in np.unique(spec.owner_moving):
                cs = [tuple(As[1:4, c]) for c in range(As.shape[1])
                      if As[0, c] == Q_ and spec.owner_static[As[2, c], As[1, c]] == P_]
                cm = []
                for c in range(Am.shape[1]):
                    if Am[0, c] != P_:
                        continue
                    ip = Am[2, c]
                    jt = int(np.nonzero(spec.face_id_moving[ip] == Am[4, c])[0][0])
                    if spec.owner_moving[ip, jt] == Q_:
                        cm.append(tuple(Am[1:4, c]))
                assert cs == cm

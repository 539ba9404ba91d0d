"""GPU: the BR1 lifting surface term (mortar_lifting) against the FP64 oracle, element
by element per output plane (3 normal components x 5 variables), at sizes that span
several tiles and a ragged tail, with per-point metrics, over degrees 1-15 (FP32 up to
degree 9 runs the register-direct lifting body, the rest the VALU lifting kernel), tiny
periodic rows, and the plane N=5 workload's shape at full size, every row."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

from . import _parity as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2008_04356_amd import mortar
    return mortar


def _alloc(spec):
    import torch
    dt = H.torch_dtype(spec.precision)
    Ls = torch.full((3, 5, spec.P, spec.n_face_static), float("nan"), dtype=dt, device="cuda:0")
    Lm = torch.full((3, 5, spec.P, spec.n_face_moving), float("nan"), dtype=dt, device="cuda:0")
    return Ls, Lm


def _err(spec, got, ref, rows=None):
    """Per output plane (component c, variable v): max |difference| over the interface's
    columns of both sides, relative to the plane's largest reference value, floored at
    1e-3 of the largest over all planes (components along zero normal entries are 0)."""
    fs, fm = spec.face_id_static, spec.face_id_moving
    if rows is not None:
        fs, fm = fs[rows[0]:rows[1]], fm[rows[0]:rows[1]]
    cs, cm = fs.ravel(), fm.ravel()
    g = [np.asarray(got[0], dtype=np.float64)[:, :, :, cs], np.asarray(got[1], dtype=np.float64)[:, :, :, cm]]
    r = [ref[0][:, :, :, cs], ref[1][:, :, :, cm]]
    scale = np.maximum(np.max(np.abs(r[0]), axis=(2, 3)), np.max(np.abs(r[1]), axis=(2, 3)))
    floor = 1e-3 * np.max(scale)
    diff = np.maximum(np.max(np.abs(g[0] - r[0]), axis=(2, 3)), np.max(np.abs(g[1] - r[1]), axis=(2, 3)))
    return (diff / np.maximum(scale, floor)).ravel()


def _case(M, spec, disps, seed=3, noise=1e-3, rows=None):
    import torch
    op = M.MortarOperator([spec])
    inp = W.make_inputs(spec, seed=seed, delta=disps[0], noise=noise)
    din, oin = H.device_inputs(spec, inp), H.oracle_inputs(spec, inp)
    try:
        for d in disps:
            print(f"[lifting] N={spec.N} {spec.n_par}x{spec.n_perp} prec={spec.precision} "
                  f"met={spec.metrics is not None} disp={d:.6g}", flush=True)
            op.update([d])
            n, s = O.decompose(d, spec.l_par)
            Ls, Lm = _alloc(spec)
            op.lifting([din["Us"]], [din["Um"]], [Ls], [Lm])
            torch.cuda.synchronize()
            got = (Ls.cpu().numpy(), Lm.cpu().numpy())
            ref = O.mortar_lifting(spec, n, s, oin["Us"], oin["Um"], rows=rows, threads=H.oracle_threads())
            err = _err(spec, got, ref, rows=rows)
            assert np.max(err) <= H.TOL[spec.precision], (d, err)
            for L, fid, nf in ((got[0], spec.face_id_static, spec.n_face_static),
                               (got[1], spec.face_id_moving, spec.n_face_moving)):
                off = np.setdiff1d(np.arange(nf), fid.ravel())
                if off.size:
                    assert np.all(np.isnan(L[:, :, :, off]))
    finally:
        op.close()


@pytest.mark.parametrize("precision", [W.FP64, W.FP32])
def test_plane_multi_tile_ragged(M, precision):
    spec = W.make_plane(5, 70, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=precision,
                        scramble_seed=2, extra_cols=3)
    _case(M, spec, [0.3137 * spec.l_par, 17.77 * spec.l_par, 0.0])


@pytest.mark.parametrize("precision", [W.FP64, W.FP32])
def test_annulus_metrics(M, precision):
    spec = W.make_annulus(7, 40, 3, seed=3, precision=precision)
    _case(M, spec, [0.37 * spec.l_par, 11.5 * spec.l_par])


@pytest.mark.parametrize("N,node_set", [(1, W.GAUSS), (2, W.LGL), (3, W.GAUSS), (4, W.LGL),
                                        (6, W.GAUSS), (8, W.LGL), (9, W.GAUSS), (10, W.GAUSS),
                                        (12, W.LGL), (15, W.GAUSS)])
def test_degrees(M, N, node_set):
    spec = W.make_plane(N, 23, 2, physics=W.EULER, riemann=W.ROE, node_set=node_set,
                        precision=W.FP32, scramble_seed=N, extra_cols=1)
    _case(M, spec, [0.41 * spec.l_par, 5.003 * spec.l_par], seed=N)


@pytest.mark.parametrize("n_par", [1, 2, 3, 16])
def test_tiny_and_single_tile_rows(M, n_par):
    """Rows of 1-3 faces (a tile wraps around the periodic row) and of one tile plus one
    face, FP32 degree 3: the register-direct lifting body."""
    spec = W.make_plane(3, n_par, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32,
                        scramble_seed=n_par, extra_cols=1)
    _case(M, spec, [0.3 * spec.l_par, 2.7 * spec.l_par, 41.05 * spec.l_par], seed=n_par)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_annulus_metrics_fp32_degrees(M, N):
    """Per-point metrics in FP32 over the degrees of both lifting kernels (register-direct
    up to degree 9, VALU from 10), including those whose 2 (N + 1) mortar nodes leave
    padding rows in a register that holds real nodes too (N = 2, 4, 6, 8): a padding
    row's normal is not finite and must not reach the outputs."""
    spec = W.make_annulus(N, 37, 3, seed=N, precision=W.FP32)
    _case(M, spec, [0.2 * spec.l_par, 9.7 * spec.l_par], seed=N)


def test_plane_workload_full_size_all_rows(M):
    specs, disp = W.config(2, precision=W.FP32)
    _case(M, specs[0], [disp(137)[0]], seed=2, noise=1e-4)


def test_not_ready_before_update(M):
    spec = W.make_plane(3, 8, 1, precision=W.FP32)
    op = M.MortarOperator([spec])
    try:
        din = H.device_inputs(spec, W.make_inputs(spec, seed=1))
        Ls, Lm = _alloc(spec)
        with pytest.raises(M.MortarError, match="no displacement"):
            op.lifting([din["Us"]], [din["Um"]], [Ls], [Lm])
    finally:
        op.close()

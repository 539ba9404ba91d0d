"""GPU: the launch autotuner and explicit tunings.  Every variant and tile length must
give oracle-matching fluxes; within one variant the result may not depend on the tile
length at all (each mortar's flux and each face's sums are formed in the same order);
graphs captured before a retune are refused; the JSON cache round-trips."""
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


def _same(a, b):
    import torch
    return torch.allclose(a, b, rtol=0, atol=0, equal_nan=True)


def _setup(M, specs, disp, seed=3):
    op = M.MortarOperator(specs)
    inps = [W.make_inputs(s, seed=seed + i, delta=disp[i], noise=1e-3) for i, s in enumerate(specs)]
    dins = [H.device_inputs(s, x) for s, x in zip(specs, inps)]
    oins = [H.oracle_inputs(s, x) for s, x in zip(specs, inps)]
    op.update(disp)
    return op, dins, oins


def _args(dins, outs):
    return ([d["Us"] for d in dins], [d["Um"] for d in dins], [d["Gs"] for d in dins],
            [d["Gm"] for d in dins], [o[0] for o in outs], [o[1] for o in outs])


def test_single_interface_every_variant_and_tile(M):
    spec = W.make_plane(5, 47, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32,
                        scramble_seed=2, extra_cols=1)
    disp = [3.41 * spec.l_par]
    op, dins, oins = _setup(M, [spec], disp)
    try:
        n, s = O.decompose(disp[0], spec.l_par)
        ref = H.oracle_flux(spec, oins[0], n, s)
        per_variant = {}
        for variant in (M.KERNEL_VALU, M.KERNEL_MFMA_LDS, M.KERNEL_REGISTER, M.KERNEL_VALU_WIDE,
                        M.KERNEL_HYBRID):
            for tile in (0, 11, 6, 3):
                print(f"[autotune] variant={variant} tile={tile}", flush=True)
                assert M.mortar_set_tuning(op.h, 0, variant, tile, 0) == 0
                outs = H.gpu_flux(op, [spec], dins)
                err = H.rel_err(spec, (outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy()), ref)
                assert np.max(err) <= H.TOL[W.FP32], (variant, tile, err)
                if variant in per_variant:
                    assert _same(outs[0][0], per_variant[variant][0])
                    assert _same(outs[0][1], per_variant[variant][1])
                else:
                    per_variant[variant] = outs[0]
        # explicit grid sizes (persistent launch with fewer workgroups)
        assert M.mortar_set_tuning(op.h, 0, M.KERNEL_VALU, 0, 8) == 0
        outs = H.gpu_flux(op, [spec], dins)
        assert _same(outs[0][0], per_variant[M.KERNEL_VALU][0])
        chosen = op.autotune(*_args(dins, H.gpu_flux(op, [spec], dins)), reps=2)
        assert chosen[0]["variant"] in (0, 1, 2, 3, 4)
        outs = H.gpu_flux(op, [spec], dins)
        err = H.rel_err(spec, (outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy()), ref)
        assert np.max(err) <= H.TOL[W.FP32], (chosen, err)
    finally:
        op.close()


def test_invalid_tunings(M):
    spec = W.make_plane(3, 9, 2, precision=W.BF16_MFMA)
    op, _, _ = _setup(M, [spec], [0.3 * spec.l_par])
    try:
        bad = M.mortar_set_tuning(op.h, 0, M.KERNEL_VALU, 0, 0)     # bf16 runs one variant
        assert bad == -1
        assert M.mortar_set_tuning(op.h, 0, M.KERNEL_REGISTER, 0, 3) == -1   # grid < 8
        assert M.mortar_set_tuning(op.h, 0, 7, 0, 0) == -1
        assert M.mortar_set_tuning(op.h, 1, M.KERNEL_REGISTER, 0, 0) == -1   # no such iface
        assert M.mortar_set_tuning(op.h, 0, M.KERNEL_REGISTER, 5, 64) == 0
        assert op.tuning()[0] == {"variant": 2, "tile_len": 5, "grid": 64}
    finally:
        op.close()


def test_batched_tuning_graph_and_cache(M, tmp_path):
    import torch
    specs = [W.make_annulus(7, 40, 3, seed=11, precision=W.FP32, name="a7"),
             W.make_annulus(5, 33, 2, seed=12, precision=W.FP32, name="a5"),
             W.make_plane(3, 17, 4, physics=W.NS, riemann=W.ROE, mu=1e-4, precision=W.FP32,
                          name="p3")]
    disp = [0.7 * s.l_par for s in specs]
    op, dins, oins = _setup(M, specs, disp)
    try:
        base = H.gpu_flux(op, specs, dins)
        outs = [H.alloc_outputs(s) for s in specs]
        g = op.graph(*_args(dins, outs))
        cache = str(tmp_path / "tune.json")
        chosen = op.autotune(*_args(dins, [H.alloc_outputs(s) for s in specs]), reps=2,
                             cache=cache)
        # one kernel for the whole batch: VALU or register-direct (N = 3, 5, 7 in FP32)
        assert len({c["variant"] for c in chosen}) == 1
        assert chosen[0]["variant"] in (M.KERNEL_VALU, M.KERNEL_REGISTER)
        tuned = H.gpu_flux(op, specs, dins)
        if chosen[0]["variant"] == M.KERNEL_VALU:   # same kernel, other tiles: same bits
            for a, b in zip(base, tuned):
                assert _same(a[0], b[0]) and _same(a[1], b[1])
        # the graph was captured before the retune: refused until captured again
        with pytest.raises(M.MortarError):
            g.launch(disp)
        g.close()
        g = op.graph(*_args(dins, outs))
        g.launch(disp)
        torch.cuda.synchronize()
        for a, b in zip(tuned, outs):
            assert _same(a[0], b[0]) and _same(a[1], b[1])
        g.close()
        # oracle parity of the tuned batch
        for i, s in enumerate(specs):
            n, sf = O.decompose(disp[i], s.l_par)
            ref = H.oracle_flux(s, oins[i], n, sf)
            err = H.rel_err(s, (tuned[i][0].cpu().numpy(), tuned[i][1].cpu().numpy()), ref)
            assert np.max(err) <= H.TOL[W.FP32], (s.name, err)
        # a second operator of the same shapes takes the cached choice without timing
        op2 = M.MortarOperator(specs)
        try:
            op2.update(disp)
            got = op2.autotune(None, None, None, None, None, None, cache=cache)
            assert got == chosen and op2.tuning() == chosen
        finally:
            op2.close()
    finally:
        op.close()


def _close(a, b, rel=1e-6):
    """Equal up to a few FP32 ulps of each variable's largest value (two separately
    compiled kernels may contract multiply-adds differently)."""
    import torch
    a, b = a.double(), b.double()
    for v in range(5):
        scale = max(float(torch.nan_to_num(a[v]).abs().max()), 1e-30)
        d = torch.nan_to_num(a[v] - b[v], nan=0.0).abs().max()
        if float(d) > rel * scale or not torch.equal(torch.isnan(a[v]), torch.isnan(b[v])):
            return False
    return True


@pytest.mark.parametrize("riemann", [W.ROE, W.LF])
def test_batched_register_direct_kernel_euler(M, riemann):
    """An Euler batch of degrees 7, 5, 3 (FP32) through the batched register-direct kernel:
    its N = 7 member runs in the lockstep rounds, the others with the same eight-wave
    workgroups; every member agrees with its own register-direct launch to a few ulps and
    with the oracle to the FP32 tolerance, on two grids."""
    specs = [W.make_plane(7, 41, 3, physics=W.EULER, riemann=riemann, precision=W.FP32,
                          scramble_seed=5, extra_cols=1, name="e7"),
             W.make_plane(5, 33, 2, physics=W.EULER, riemann=riemann, precision=W.FP32, name="e5"),
             W.make_plane(3, 17, 3, physics=W.EULER, riemann=riemann, precision=W.FP32, name="e3")]
    disp = [2.3 * s.l_par for s in specs]
    op, dins, oins = _setup(M, specs, disp, seed=11)
    singles = []
    try:
        for i, s in enumerate(specs):
            o = M.MortarOperator([s])
            o.update([disp[i]])
            assert M.mortar_set_tuning(o.h, 0, M.KERNEL_REGISTER, 0, 0) == 0
            singles.append((o, H.gpu_flux(o, [s], [dins[i]])[0]))
        for grid in (0, 11):
            assert M.mortar_set_tuning(op.h, 0, M.KERNEL_REGISTER, 0, grid) == 0
            outs = H.gpu_flux(op, specs, dins)
            for i, s in enumerate(specs):
                assert _close(outs[i][0], singles[i][1][0]) and _close(outs[i][1], singles[i][1][1]), s.name
                n, sf = O.decompose(disp[i], s.l_par)
                ref = H.oracle_flux(s, oins[i], n, sf)
                err = H.rel_err(s, (outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy()), ref)
                assert np.max(err) <= H.TOL[W.FP32], (s.name, grid, err)
    finally:
        for o, _ in singles:
            o.close()
        op.close()


def test_batched_register_direct_kernel(M):
    """The batched register-direct kernel (FP32, N = 3, 5, 7) agrees with each interface's
    own register-direct launch to a few ulps, and with the oracle to the FP32 tolerance."""
    specs = [W.make_annulus(7, 37, 3, seed=21, precision=W.FP32, name="a7"),
             W.make_annulus(5, 30, 2, seed=22, precision=W.FP32, name="a5"),
             W.make_plane(3, 19, 3, physics=W.NS, riemann=W.ROE, mu=1e-4, precision=W.FP32,
                          scramble_seed=3, extra_cols=2, name="p3")]
    disp = [1.3 * s.l_par for s in specs]
    op, dins, oins = _setup(M, specs, disp, seed=9)
    singles = []
    try:
        for i, s in enumerate(specs):
            o = M.MortarOperator([s])
            o.update([disp[i]])
            assert M.mortar_set_tuning(o.h, 0, M.KERNEL_REGISTER, 0, 0) == 0
            singles.append((o, H.gpu_flux(o, [s], [dins[i]])[0]))
        for tile in (0, 9):
            assert M.mortar_set_tuning(op.h, 0, M.KERNEL_REGISTER, tile, 0) == 0
            assert op.tuning()[0]["variant"] == M.KERNEL_REGISTER
            outs = H.gpu_flux(op, specs, dins)
            for i, s in enumerate(specs):
                assert _close(outs[i][0], singles[i][1][0]) and _close(outs[i][1], singles[i][1][1]), s.name
                n, sf = O.decompose(disp[i], s.l_par)
                ref = H.oracle_flux(s, oins[i], n, sf)
                err = H.rel_err(s, (outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy()), ref)
                assert np.max(err) <= H.TOL[W.FP32], (s.name, err)
        # a batch with a degree outside {3, 5, 7} has no register-direct batch kernel
        bad = M.MortarOperator([W.make_plane(4, 9, 2, physics=W.NS, riemann=W.ROE, mu=1e-4,
                                             precision=W.FP32),
                                W.make_plane(3, 9, 2, physics=W.NS, riemann=W.ROE, mu=1e-4,
                                             precision=W.FP32)])
        try:
            assert M.mortar_set_tuning(bad.h, 0, M.KERNEL_REGISTER, 0, 0) == -1
        finally:
            bad.close()
    finally:
        for o, _ in singles:
            o.close()
        op.close()

"""GPU: several interfaces with different degrees and face counts in one persistent
launch (the batched kernel) against separate single-interface launches (bitwise) and the
oracle; the per-stage HIP graph against eager launches over stages that cross faces."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

from . import _parity as H

pytestmark = pytest.mark.gpu


def same(x, y):
    """Bitwise equal, with the NaN sentinels of untouched columns equal to each other."""
    import torch
    return torch.allclose(x, y, rtol=0.0, atol=0.0, equal_nan=True)


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    from paper_2008_04356_amd import mortar
    return mortar


def _turbine_like(precision, scale=1):
    return [W.make_annulus(7, 40 * scale, 5, seed=41, precision=precision, name="b-I0"),
            W.make_annulus(5, 33 * scale, 4, seed=42, precision=precision, name="b-I1"),
            W.make_plane(3, 17 * scale, 3, physics=W.NS, riemann=W.ROE, mu=1e-3,
                         precision=precision, scramble_seed=3, extra_cols=2, name="b-I2")]


@pytest.mark.parametrize("precision", [W.FP32, W.FP64])
def test_batched_equals_single_and_oracle(M, precision):
    import torch
    specs = _turbine_like(precision)
    disps = [[0.37 * s.l_par, 2.6 * s.l_par, -1.3 * s.l_par][i] for i, s in enumerate(specs)]
    ins = [W.make_inputs(s, seed=10 + i, delta=disps[i], noise=1e-3) for i, s in enumerate(specs)]
    dins = [H.device_inputs(s, x) for s, x in zip(specs, ins)]
    print(f"[batch] precision={precision} n_if={len(specs)}", flush=True)
    op = M.MortarOperator(specs)
    try:
        op.update(disps)
        outs = H.gpu_flux(op, specs, dins)
    finally:
        op.close()
    for i, s in enumerate(specs):
        single = M.MortarOperator([s])
        try:
            single.update([disps[i]])
            ref = H.gpu_flux(single, [s], [dins[i]])
        finally:
            single.close()
        assert same(outs[i][0], ref[0][0]) and same(outs[i][1], ref[0][1]), s.name
        n, sf = O.decompose(disps[i], s.l_par)
        ora = H.oracle_flux(s, H.oracle_inputs(s, ins[i]), n, sf)
        err = H.rel_err(s, (outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy()), ora)
        assert np.max(err) <= H.TOL[precision], (s.name, err)


def test_graph_replay_equals_eager(M):
    import torch
    specs = _turbine_like(W.FP32)
    ins = [W.make_inputs(s, seed=20 + i, noise=1e-3) for i, s in enumerate(specs)]
    dins = [H.device_inputs(s, x) for s, x in zip(specs, ins)]
    speeds = [0.0137, 0.0211, 0.0093]
    op_g = M.MortarOperator(specs)
    op_e = M.MortarOperator(specs)
    try:
        outs_g = [H.alloc_outputs(s) for s in specs]
        op_g.update([0.0, 0.0, 0.0])
        graph = op_g.graph([d["Us"] for d in dins], [d["Um"] for d in dins],
                           [d["Gs"] for d in dins], [d["Gm"] for d in dins],
                           [o[0] for o in outs_g], [o[1] for o in outs_g])
        try:
            # large steps so that several stages cross whole faces (index-map rebuilds)
            for k in range(12):
                disp = [37.0 * speeds[i] * k * specs[i].l_par for i in range(3)]
                print(f"[graph] stage {k}", flush=True)
                graph.launch(disp)
                torch.cuda.synchronize()
                op_e.update(disp)
                ref = H.gpu_flux(op_e, specs, dins)
                scratch = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
                torch.cuda.synchronize()
                del scratch
                for i in range(3):
                    assert same(outs_g[i][0], ref[i][0]) and same(outs_g[i][1], ref[i][1])
                    for side in (0, 1):
                        Ag, mg = op_g.index_map(i, side)
                        Ae, me = op_e.index_map(i, side)
                        assert np.array_equal(Ag, Ae) and np.array_equal(mg, me)
        finally:
            graph.close()
    finally:
        op_g.close()
        op_e.close()


def test_mixed_precisions_fall_back_to_separate_launches(M):
    import torch
    specs = [W.make_plane(3, 20, 2, physics=W.EULER, riemann=W.LF, precision=W.FP64, name="m64"),
             W.make_plane(4, 18, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32,
                          name="m32")]
    ins = [W.make_inputs(s, seed=30 + i, noise=1e-3) for i, s in enumerate(specs)]
    dins = [H.device_inputs(s, x) for s, x in zip(specs, ins)]
    op = M.MortarOperator(specs)
    try:
        disps = [1.25 * specs[0].l_par, 0.5 * specs[1].l_par]
        op.update(disps)
        outs = H.gpu_flux(op, specs, dins)
        for i, s in enumerate(specs):
            n, sf = O.decompose(disps[i], s.l_par)
            ora = H.oracle_flux(s, H.oracle_inputs(s, ins[i]), n, sf)
            err = H.rel_err(s, (outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy()), ora)
            assert np.max(err) <= H.TOL[s.precision]
        torch.cuda.synchronize()
    finally:
        op.close()


def test_graph_replay_conservation_from_fused_partials(M):
    """A captured single-interface VALU launch writes its conservation partials on every
    replay: the sums after each replay equal a pass over copies of the flux arrays, with
    an eager launch into other buffers (and its partials) between the replays."""
    import torch
    spec = W.make_plane(5, 53, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32,
                        scramble_seed=5, extra_cols=1)
    din = H.device_inputs(spec, W.make_inputs(spec, seed=31, noise=1e-2))
    op = M.MortarOperator([spec])
    try:
        assert M.mortar_set_tuning(op.h, 0, M.KERNEL_VALU, 0, 0) == 0
        outs = [H.alloc_outputs(spec, fill=0.0)]
        other = [H.alloc_outputs(spec, fill=0.0)]
        op.update([0.0])
        graph = op.graph([din["Us"]], [din["Um"]], [din["Gs"]], [din["Gm"]],
                         [outs[0][0]], [outs[0][1]])
        try:
            for k in range(4):
                print(f"[graph] conservation stage {k}", flush=True)
                graph.launch([(0.31 + 7.7 * k) * spec.l_par])
                dev = torch.zeros((1, 5, 3), dtype=torch.float64, device="cuda:0")
                op.conservation_device([outs[0][0]], [outs[0][1]], dev)
                torch.cuda.synchronize()
                fused = dev.cpu().numpy()[0]
                passed = op.conservation([outs[0][0].clone()], [outs[0][1].clone()])[0]
                assert np.all(np.abs(fused - passed) <= 1e-13 * passed[:, 2:3] + 1e-300), (k, fused, passed)
                # an eager launch into other buffers moves the partials to those buffers
                op.update([(0.77 + 3.1 * k) * spec.l_par])
                H.gpu_flux(op, [spec], [din], outs=other)
                again = op.conservation([outs[0][0]], [outs[0][1]])[0]
                assert np.all(np.abs(again - passed) <= 1e-13 * passed[:, 2:3] + 1e-300)
        finally:
            graph.close()
    finally:
        op.close()


@pytest.mark.parametrize("which", ["fp32_batch", "fp64_single", "mixed"])
def test_graph_with_conservation_sums(M, which):
    """A stage graph holding the conservation sums (mortar_graph_create_cons): after every
    replay the sums it wrote equal, bit for bit, those an eager conservation_device call
    forms from the same flux outputs, and agree with a pass over copies of them; the
    program's own eager work runs between the replays."""
    import torch
    if which == "fp32_batch":
        specs = _turbine_like(W.FP32)
    elif which == "fp64_single":
        specs = [W.make_plane(5, 53, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP64,
                              scramble_seed=7, name="g64")]
    else:
        # element types differ: one launch per interface, each with its own sums
        specs = [W.make_plane(3, 20, 2, physics=W.EULER, riemann=W.LF, precision=W.FP64, name="m64"),
                 W.make_plane(4, 18, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32,
                              name="m32")]
    ins = [W.make_inputs(s, seed=40 + i, noise=1e-3) for i, s in enumerate(specs)]
    dins = [H.device_inputs(s, x) for s, x in zip(specs, ins)]
    op = M.MortarOperator(specs)
    try:
        outs = [H.alloc_outputs(s) for s in specs]
        cons_g = torch.zeros((len(specs), 5, 3), dtype=torch.float64, device="cuda:0")
        op.update([0.0] * len(specs))
        graph = op.graph([d["Us"] for d in dins], [d["Um"] for d in dins],
                         [d["Gs"] for d in dins], [d["Gm"] for d in dins],
                         [o[0] for o in outs], [o[1] for o in outs], cons_out=cons_g)
        try:
            for k in range(6):
                # steps of several faces, so that some stages rebuild the index maps
                disp = [(0.37 + 5.3 * k) * s.l_par for s in specs]
                print(f"[graph+cons] {which} stage {k}", flush=True)
                graph.launch(disp)
                torch.cuda.synchronize()
                got = cons_g.cpu().numpy().copy()
                ref = torch.zeros_like(cons_g)
                op.conservation_device([o[0] for o in outs], [o[1] for o in outs], ref)
                scratch = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
                torch.cuda.synchronize()
                del scratch
                assert np.array_equal(got, ref.cpu().numpy()), (k, got, ref)
                passed = np.array(op.conservation([o[0].clone() for o in outs],
                                                  [o[1].clone() for o in outs]))
                assert np.all(np.abs(got - passed) <= 1e-13 * passed[:, :, 2:3] + 1e-300), (k, got, passed)
                assert np.all(passed[:, :, 2] > 0)
        finally:
            graph.close()
    finally:
        op.close()


def test_graph_with_conservation_rejects_missing_output(M):
    specs = _turbine_like(W.FP32)
    dins = [H.device_inputs(s, W.make_inputs(s, seed=50 + i, noise=1e-3)) for i, s in enumerate(specs)]
    op = M.MortarOperator(specs)
    try:
        outs = [H.alloc_outputs(s) for s in specs]
        op.update([0.0] * len(specs))
        p = lambda ts: [t.data_ptr() for t in ts]  # noqa: E731
        with pytest.raises(M.MortarError):
            M.mortar_graph_create_cons(op.h, p([d["Us"] for d in dins]), p([d["Um"] for d in dins]),
                                       p([d["Gs"] for d in dins]), p([d["Gm"] for d in dins]),
                                       p([o[0] for o in outs]), p([o[1] for o in outs]), 0)
    finally:
        op.close()

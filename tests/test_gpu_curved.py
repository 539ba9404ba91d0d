"""GPU: curved interfaces (cylindrical radial and conical surfaces of revolution with
polynomial face geometry, per-point static metrics whose normal turns along the slide)
against the FP64 oracle: the flux in every launch variant, over degrees, the BR1 lifting
term, a batch of curved and flat interfaces in one launch, the bf16/fp16 modes, and the
full-size curved workloads on every row."""
import math

import numpy as np
import pytest

from paper_2008_04356_amd import workloads as W

from .test_gpu_batch import same
from .test_gpu_lifting import _case as lifting_case
from .test_gpu_lowprec import _lowprec_case
from .test_gpu_parity import _VARIANTS, _run_and_compare
from . import _parity as H

pytestmark = pytest.mark.gpu

SHAPES = {"cylinder": 0.0, "cone": math.pi / 5}


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2008_04356_amd import mortar
    return mortar


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("precision,variant",
                         [(p, v) for p in (W.FP32, W.FP64) for v in _VARIANTS[p]])
def test_variants(M, shape, precision, variant):
    # 37 faces per row: several tiles and a ragged tail in every variant
    spec = W.make_revolution(5, 37, 3, SHAPES[shape], seed=5, precision=precision,
                             mu=1e-3, name=shape)
    _run_and_compare(M, spec, [0.37 * spec.l_par, 11.5 * spec.l_par], seed=4, noise=1e-3,
                     check_maps=False, variant=variant)


@pytest.mark.parametrize("N,node_set,shape", [(1, W.GAUSS, "cylinder"), (3, W.LGL, "cone"),
                                              (7, W.GAUSS, "cone"), (9, W.LGL, "cylinder")])
@pytest.mark.parametrize("precision", [W.FP32, W.FP64])
def test_degrees(M, N, node_set, shape, precision):
    spec = W.make_revolution(N, 23, 2, SHAPES[shape], seed=N, node_set=node_set,
                             precision=precision, mu=1e-3, name=shape)
    _run_and_compare(M, spec, [0.41 * spec.l_par, 5.003 * spec.l_par], seed=N, noise=1e-3,
                     check_maps=False)


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("precision", [W.FP32, W.FP64])
def test_lifting(M, shape, precision):
    spec = W.make_revolution(5, 37, 3, SHAPES[shape], seed=8, precision=precision, name=shape)
    lifting_case(M, spec, [0.37 * spec.l_par, 11.5 * spec.l_par])


@pytest.mark.parametrize("precision", [W.FP32, W.FP64])
def test_batch_of_curved_and_flat(M, precision):
    from oracle import oracle as O
    specs = [W.make_revolution(7, 40, 4, 0.0, seed=41, precision=precision, name="b-cyl"),
             W.make_revolution(5, 33, 3, math.pi / 6, seed=42, precision=precision, name="b-cone"),
             W.make_plane(3, 17, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=precision,
                          scramble_seed=3, extra_cols=2, name="b-plane")]
    disps = [0.37 * specs[0].l_par, 2.6 * specs[1].l_par, -1.3 * specs[2].l_par]
    ins = [W.make_inputs(s, seed=10 + i, delta=disps[i], noise=1e-3) for i, s in enumerate(specs)]
    dins = [H.device_inputs(s, x) for s, x in zip(specs, ins)]
    print(f"[curved batch] precision={precision}", flush=True)
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


@pytest.mark.parametrize("precision", [W.BF16_MFMA, W.FP16_MFMA])
def test_lowprec_cone(M, precision):
    spec = W.make_revolution(5, 24, 3, SHAPES["cone"], seed=7, precision=precision)
    # the derived per-variable bound is asserted inside the case
    _lowprec_case(M, spec, [0.2 * spec.l_par, 3.7 * spec.l_par])


@pytest.mark.parametrize("config,precision,variant",
                         [(6, W.FP32, v) for v in _VARIANTS[W.FP32]]
                         + [(6, W.FP64, None), (7, W.FP32, None), (7, W.FP64, None)])
def test_full_size_all_rows(M, config, precision, variant):
    """The curved workloads (N=7, 512x64) at full size, every row against the oracle."""
    specs, disp = W.config(config, precision=precision)
    _run_and_compare(M, specs[0], [disp(211)[0]], seed=3, noise=1e-4, check_maps=False,
                     variant=variant)

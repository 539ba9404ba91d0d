"""GPU: projection GEMMs with bf16 / fp16 operands (FP32 data and accumulation) and the
conservation-corrected back projection, against the FP64 oracle.

The oracle sees the same FP32 inputs in FP64.  Rounding the GEMM operands to a format
with unit roundoff u (bf16 2^-9, fp16 2^-12 for round-to-nearest) perturbs each
projected value by about u times the sum of |P| |operand| (the Lebesgue-type sums of the
sub-interval interpolation stay below 3 for N <= 9), once forward and once backward, and
the Riemann flux passes this on with O(1) amplification for the smooth states used here.
The bounds below are 64 u: loose enough for every variable of these states and still far
below what a wrong matrix, index or sign gives (an O(1) error)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

from . import _parity as H

pytestmark = pytest.mark.gpu

U_ROUND = {W.BF16_MFMA: 2.0 ** -9, W.FP16_MFMA: 2.0 ** -12}


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2008_04356_amd import mortar
    return mortar


def _lowprec_case(M, spec, disps, seed=5):
    op = M.MortarOperator([spec])
    inp = W.make_inputs(spec, seed=seed, delta=disps[0], noise=1e-3)
    din, oin = H.device_inputs(spec, inp), H.oracle_inputs(spec, inp)
    errs = []
    try:
        for d in disps:
            print(f"[lowprec] N={spec.N} {spec.n_par}x{spec.n_perp} prec={spec.precision} "
                  f"phys={spec.physics} disp={d:.6g}", flush=True)
            op.update([d])
            n, s = O.decompose(d, spec.l_par)
            outs = H.gpu_flux(op, [spec], [din])
            Fs, Fm = outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy()
            ref = H.oracle_flux(spec, oin, n, s)
            err = H.rel_err(spec, (Fs, Fm), ref)
            errs.append(err)
            assert np.all(np.isfinite(err)), err
            assert np.max(err) <= 64 * U_ROUND[spec.precision], (d, err)
            # line-by-line correction: the static and moving integrals agree to FP32
            # storage rounding, as in the FP32 mode
            c = op.conservation([outs[0][0]], [outs[0][1]])[0]
            assert np.all(np.abs(c[:, 0] - c[:, 1]) <= 2e-6 * c[:, 2]), c
            for F, fid, nf in ((Fs, spec.face_id_static, spec.n_face_static),
                               (Fm, spec.face_id_moving, spec.n_face_moving)):
                off = np.setdiff1d(np.arange(nf), fid.ravel())
                if off.size:
                    assert np.all(np.isnan(F[:, :, off]))
    finally:
        op.close()
    return np.max(np.array(errs), axis=0)


@pytest.mark.parametrize("precision", [W.BF16_MFMA, W.FP16_MFMA])
def test_c5_shape_euler_roe(M, precision):
    """N = 9 plane, Euler + Roe (the precision-stress workload's physics), several tiles
    per row with a ragged tail, scrambled columns."""
    spec = W.make_plane(9, 37, 3, physics=W.EULER, riemann=W.ROE, precision=precision,
                        scramble_seed=9, extra_cols=3)
    err = _lowprec_case(M, spec, [0.0, 0.37 * spec.l_par, 5.81 * spec.l_par, 36.5 * spec.l_par])
    print(f"[lowprec] per-variable error {precision}: {err}", flush=True)


@pytest.mark.parametrize("precision", [W.BF16_MFMA, W.FP16_MFMA])
@pytest.mark.parametrize("N,physics", [(3, W.EULER), (5, W.NS), (7, W.NS)])
def test_degrees_and_physics(M, precision, N, physics):
    spec = W.make_plane(N, 19, 2, physics=physics, riemann=W.ROE,
                        mu=1e-3 if physics == W.NS else 0.0, precision=precision)
    _lowprec_case(M, spec, [0.61 * spec.l_par, 11.2 * spec.l_par])


@pytest.mark.parametrize("precision", [W.BF16_MFMA, W.FP16_MFMA])
def test_annulus_metrics_lowprec(M, precision):
    spec = W.make_annulus(5, 24, 3, seed=7, precision=precision)
    _lowprec_case(M, spec, [0.2 * spec.l_par, 3.7 * spec.l_par])


@pytest.mark.parametrize("precision,variant", [(W.BF16_MFMA, 2), (W.FP16_MFMA, 2)])
def test_c5_full_size_sampled_rows(M, precision, variant):
    """The precision-stress workload at full size (plane N = 9, 256 x 256; surface
    elements of 3.8e-6 put the fluxes far below fp16's normal range before scaling);
    the oracle checks three rows."""
    specs, disp = W.config(5, precision=precision)
    spec = specs[0]
    d = disp(37)[0]
    op = M.MortarOperator([spec])
    try:
        assert M.mortar_set_tuning(op.h, 0, variant, 0, 0) == 0
        inp = W.make_inputs(spec, seed=2, delta=d, noise=1e-4)
        din, oin = H.device_inputs(spec, inp), H.oracle_inputs(spec, inp)
        op.update([d])
        n, s = O.decompose(d, spec.l_par)
        outs = H.gpu_flux(op, [spec], [din])
        rows = (101, 104)
        ref = H.oracle_flux(spec, oin, n, s, rows=rows)
        err = H.rel_err(spec, (outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy()), ref, rows=rows)
        print(f"[lowprec] plane N=9 256x256 full size {precision}: per-variable error {err}", flush=True)
        assert np.max(err) <= 64 * U_ROUND[precision], err
        c = op.conservation([outs[0][0]], [outs[0][1]])[0]
        assert np.all(np.abs(c[:, 0] - c[:, 1]) <= 2e-6 * c[:, 2]), c
    finally:
        op.close()

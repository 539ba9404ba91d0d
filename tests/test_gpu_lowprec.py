"""GPU: projection GEMMs with bf16 / fp16 operands (FP32 data and accumulation) and the
conservation-corrected back projection, against the FP64 oracle.

The oracle sees the same FP32 inputs in FP64.  The error bound of each output variable
is derived from the arithmetic (see lowprec_bound): round-to-nearest to p significant
bits (bf16 p = 8, fp16 p = 11) has unit roundoff u = 2^-p, and both the matrices and the
operands of each projection GEMM are rounded; the forward error reaches the flux through
its Jacobian (measured on the test's own states), and the back projection adds its own
rounding and the per-line correction."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

from . import _parity as H

pytestmark = pytest.mark.gpu

U_ROUND = {W.BF16_MFMA: 2.0 ** -8, W.FP16_MFMA: 2.0 ** -11}


def lowprec_bound(spec, oin, n, s, ref, u):
    """Per-variable bound of the R15-normalised error of a bf16/fp16 projection run.

    Forward: a mortar value q = sum_j Pf_kj x_j computed with both Pf_kj and x_j rounded
    (relative u each, FP32 accumulation) is off by at most 2 u sum_j |Pf_kj| |x_j| <=
    2 u Lf max|x|, Lf = the largest row sum of |Pf| over the four sub-interval matrices
    (computed from the matrices of this s).  The flux passes these errors on through its
    Jacobians: |dF_v| <= sum_w (|dF_v/dqL_w| + |dF_v/dqR_w|) 2 u Lf max|x_w|, with the
    Jacobian sums the largest over sampled states of the test (and the per-point metrics,
    when present, add 2 u Lf |F_v| for the projected surface element).  Backward: a face
    value sum_k,q Pb_k,jq F_kq with Pb and F rounded adds 2 u Lb max|F_v| and passes the
    flux error on with Lb, Lb = the largest row sum of |Pb| over the two matrices of a
    face; the per-line correction (T - A)/sum(w) moves a value by at most the line's
    weighted mean rounding error of A, another u-sized term bounded by 2 u Lb max|F_v|."""
    mats = O.projection_matrices(spec.N, spec.node_set, s)
    Pf, Pb = mats["Pf"], mats["Pb"]
    Lf = float(np.max(np.abs(Pf).sum(axis=2)))
    Lb = float(max(np.max(np.abs(Pb[0]).sum(axis=1) + np.abs(Pb[1]).sum(axis=1)),
                   np.max(np.abs(Pb[2]).sum(axis=1) + np.abs(Pb[3]).sum(axis=1))))
    nvar = 20 if spec.physics == W.NS else 5
    cs, cm = spec.face_id_static.ravel(), spec.face_id_moving.ravel()
    xmax = np.zeros(nvar)
    for key, cols in (("Us", cs), ("Um", cm)):
        xmax[:5] = np.maximum(xmax[:5], np.abs(oin[key][:, :, cols]).max(axis=(1, 2)))
    if nvar == 20:
        for key, cols in (("Gs", cs), ("Gm", cm)):
            g = np.abs(oin[key][:, :, :, cols]).max(axis=(2, 3)).ravel()
            xmax[5:] = np.maximum(xmax[5:], g)
    J = jacobian_sums(spec, oin)
    Fmax = np.array([max(np.abs(ref[0][v][:, cs]).max(), np.abs(ref[1][v][:, cm]).max()) for v in range(5)])
    dq = 2 * u * Lf * xmax
    dF_star = J @ dq
    if spec.metrics is not None:
        dF_star = dF_star + 2 * u * Lf * Fmax
    absb = Lb * dF_star + 2 * (2 * u * Lb * Fmax)
    floor = 1e-3 * Fmax.max()
    return absb / np.maximum(Fmax, floor)


def jacobian_sums(spec, oin, n_samples=48, seed=0):
    """sum over both sides of |dF_v/dq_w| for every output variable v and projected input
    w (5 states, then 15 gradients for Navier-Stokes), the largest over face points sampled
    from the test's own inputs: central differences of the oracle's point flux, with the
    normal and surface element of the sampled point."""
    rng = np.random.default_rng(seed)
    nvar = 20 if spec.physics == W.NS else 5
    P = spec.P
    cs, cm = spec.face_id_static.ravel(), spec.face_id_moving.ravel()
    J = np.zeros((5, nvar))
    for _ in range(n_samples):
        p = int(rng.integers(P))
        a, b = int(cs[rng.integers(cs.size)]), int(cm[rng.integers(cm.size)])
        qL = np.concatenate([oin["Us"][:, p, a]] + ([oin["Gs"][:, :, p, a].ravel()] if nvar == 20 else []))
        qR = np.concatenate([oin["Um"][:, p, b]] + ([oin["Gm"][:, :, p, b].ravel()] if nvar == 20 else []))
        if spec.metrics is not None:
            nrm = spec.metrics[:3, p, a] / np.linalg.norm(spec.metrics[:3, p, a])
            dS = float(np.abs(spec.metrics[3]).max())
        else:
            nrm, dS = np.asarray(spec.normal, dtype=np.float64), spec.dS

        def F(x, y):
            return O.point_flux(x[:5], y[:5], x[5:] if nvar == 20 else None,
                                y[5:] if nvar == 20 else None, normal=nrm, dS=dS,
                                physics=spec.physics, riemann=spec.riemann, gamma=spec.gamma,
                                mu=spec.mu, Pr=spec.Pr)
        here = np.zeros((5, nvar))
        for w in range(nvar):
            e = np.zeros(nvar)
            e[w] = 1e-6 * max(1.0, abs(qL[w]), abs(qR[w]))
            here[:, w] = (np.abs(F(qL + e, qR) - F(qL - e, qR)) + np.abs(F(qL, qR + e) - F(qL, qR - e))) \
                / (2 * e[w])
        J = np.maximum(J, here)
    return J


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
    u = U_ROUND[spec.precision]
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
            bound = lowprec_bound(spec, oin, n, s, ref, u)
            print(f"[lowprec] error / derived bound per variable: {err / bound}", flush=True)
            assert np.all(err <= bound), (d, err, bound)
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
        bound = lowprec_bound(spec, oin, n, s, ref, U_ROUND[precision])
        print(f"[lowprec] plane N=9 256x256 full size {precision}: per-variable error {err}, "
              f"error / derived bound {err / bound}", flush=True)
        assert np.all(err <= bound), (err, bound)
        c = op.conservation([outs[0][0]], [outs[0][1]])[0]
        assert np.all(np.abs(c[:, 0] - c[:, 1]) <= 2e-6 * c[:, 2]), c
    finally:
        op.close()

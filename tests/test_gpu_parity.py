"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs, element by element, at sizes that span several tiles and a ragged tail; index
maps bit-exact; the full-size benchmark workload on sampled rows."""
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


def _run_and_compare(M, spec, disps, seed=1, noise=1e-3, rows=None, check_maps=True,
                     variant=None, tile=0):
    op = M.MortarOperator([spec])
    if variant is not None:
        assert M.mortar_set_tuning(op.h, 0, variant, tile, 0) == 0
    inp = W.make_inputs(spec, seed=seed, delta=disps[0], noise=noise)
    din, oin = H.device_inputs(spec, inp), H.oracle_inputs(spec, inp)
    worst = 0.0
    try:
        for d in disps:
            print(f"[parity] {spec.name or 'spec'} N={spec.N} {spec.n_par}x{spec.n_perp} "
                  f"prec={spec.precision} disp={d:.6g}", flush=True)
            op.update([d])
            n, s = O.decompose(d, spec.l_par)
            assert op.displacement(0) == (n, s)
            outs = H.gpu_flux(op, [spec], [din])
            Fs, Fm = (outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy())
            ref = H.oracle_flux(spec, oin, n, s, rows=rows)
            err = H.rel_err(spec, (Fs, Fm), ref, rows=rows)
            worst = max(worst, float(np.max(err)))
            assert np.max(err) <= H.TOL[spec.precision], (d, err)
            # columns that are not on the interface stay untouched
            for F, fid, nf in ((Fs, spec.face_id_static, spec.n_face_static),
                               (Fm, spec.face_id_moving, spec.n_face_moving)):
                off = np.setdiff1d(np.arange(nf), fid.ravel())
                if off.size:
                    assert np.all(np.isnan(F[:, :, off]))
            if check_maps:
                for side in (0, 1):
                    A, m = op.index_map(0, side)
                    own = spec.owner_moving if side == 0 else spec.owner_static
                    fid = spec.face_id_static if side == 0 else spec.face_id_moving
                    nf = spec.n_face_static if side == 0 else spec.n_face_moving
                    Ao, mo = O.index_map(side, spec.n_par, spec.n_perp, n, fid, nf, own)
                    assert np.array_equal(A, Ao) and np.array_equal(m, mo)
    finally:
        op.close()
    return worst


def test_c1_euler_lf_fp64_ten_stages(M):
    specs, disp = W.config(1)
    spec = specs[0]
    W.seeded_owners(spec, seed=1, n_static_ranks=2, n_moving_ranks=3)
    _run_and_compare(M, spec, [disp(k)[0] for k in range(10)], seed=1, noise=1e-4)


@pytest.mark.parametrize("precision", [W.FP64, W.FP32])
def test_ns_roe_multi_tile_ragged(M, precision):
    # 70 faces along the slide: several tiles and a ragged last tile in both precisions
    spec = W.make_plane(5, 70, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=precision,
                        scramble_seed=2, extra_cols=5, name="ns-ragged")
    W.seeded_owners(spec, seed=3, n_static_ranks=4, n_moving_ranks=5)
    disps = [0.3137 * spec.l_par, 17.77 * spec.l_par, -3.25 * spec.l_par, 0.0, 69.0 * spec.l_par]
    _run_and_compare(M, spec, disps, seed=7, noise=1e-3)


# every launch variant the autotuner may pick: VALU, MFMA-LDS, register-direct, and
# (FP32 only) wide-tile VALU and matrix-core-projection hybrid
_VARIANTS = {W.FP32: (0, 1, 2, 3, 4), W.FP64: (0, 1, 2)}

_DEGREE_CASES = [
    (1, W.GAUSS, W.EULER, W.ROE), (2, W.LGL, W.NS, W.ROE), (3, W.LGL, W.EULER, W.LF),
    (4, W.GAUSS, W.NS, W.LF), (6, W.GAUSS, W.EULER, W.ROE), (7, W.LGL, W.NS, W.ROE),
    (8, W.GAUSS, W.EULER, W.LF), (9, W.GAUSS, W.NS, W.ROE)]


@pytest.mark.parametrize("precision,variant,N,node_set,physics,riemann",
                         [(p, v) + c for p in (W.FP64, W.FP32) for v in _VARIANTS[p]
                          for c in _DEGREE_CASES
                          if not (v == 4 and c[0] == 9 and c[2] == W.NS)])
def test_degrees_node_sets_and_fluxes(M, precision, variant, N, node_set, physics, riemann):
    """Degrees 1-9 over both node sets, both physics and both Riemann solvers, in every
    launch variant that can take the interface (the hybrid kernel's LDS tile does not fit
    degree 9 with Navier-Stokes gradients; that refusal is tested separately)."""
    spec = W.make_plane(N, 23, 2, physics=physics, riemann=riemann, node_set=node_set,
                        mu=1e-3 if physics == W.NS else 0.0, precision=precision,
                        scramble_seed=N, extra_cols=1, name="degree")
    _run_and_compare(M, spec, [0.41 * spec.l_par, 5.003 * spec.l_par], seed=N, noise=1e-3,
                     check_maps=False, variant=variant)


@pytest.mark.parametrize("precision", [W.FP64, W.FP32])
@pytest.mark.parametrize("N,node_set,physics,riemann,annulus", [
    (10, W.LGL, W.NS, W.ROE, False), (11, W.GAUSS, W.EULER, W.LF, False),
    (12, W.GAUSS, W.NS, W.ROE, True), (13, W.LGL, W.EULER, W.ROE, False),
    (14, W.GAUSS, W.NS, W.LF, False), (15, W.GAUSS, W.NS, W.ROE, True),
    (15, W.LGL, W.EULER, W.ROE, False)])
def test_high_degrees(M, precision, N, node_set, physics, riemann, annulus):
    """Degrees 10-15 (the VALU-projection kernel, the only one built for them): several
    tiles per row and a ragged last one, scrambled columns, per-point metrics."""
    mu = 1e-3 if physics == W.NS else 0.0
    if annulus:
        spec = W.make_annulus(N, 17, 2, seed=N, physics=physics, riemann=riemann,
                              node_set=node_set, mu=mu, precision=precision, name="high-annulus")
    else:
        spec = W.make_plane(N, 17, 2, physics=physics, riemann=riemann, node_set=node_set, mu=mu,
                            precision=precision, scramble_seed=N, extra_cols=1, name="high")
    _run_and_compare(M, spec, [0.41 * spec.l_par, 5.003 * spec.l_par, -3.7 * spec.l_par],
                     seed=N, noise=1e-3, check_maps=(N == 15))


def test_high_degrees_refuse_other_variants(M):
    """Above degree 9 every variant but the VALU one, the bf16/fp16 modes and batching
    are refused or not used; degree 16 is refused."""
    spec = W.make_plane(12, 9, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32)
    op = M.MortarOperator([spec])
    try:
        for v in (1, 2, 3, 4):
            assert M.mortar_set_tuning(op.h, 0, v, 0, 0) == M.ERR_INVALID_ARG
        assert M.mortar_set_tuning(op.h, 0, 0, 0, 0) == M.OK
    finally:
        op.close()
    for prec in (W.BF16_MFMA, W.FP16_MFMA):
        lp = W.make_plane(10, 9, 2, physics=W.EULER, riemann=W.ROE, precision=prec)
        assert M.mortar_validate([M.make_desc(lp)]) == M.ERR_UNSUPPORTED
    bad = W.make_plane(16, 9, 2, physics=W.EULER, riemann=W.ROE, precision=W.FP64)
    assert M.mortar_validate([M.make_desc(bad)]) == M.ERR_UNSUPPORTED
    # a handle with a high degree launches its interfaces one by one
    a = W.make_plane(11, 9, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32)
    b = W.make_plane(3, 9, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32)
    op = M.MortarOperator([a, b])
    try:
        assert [t["variant"] for t in op.tuning()] == [0, 0]
    finally:
        op.close()


@pytest.mark.parametrize("precision", [W.FP64, W.FP32])
def test_annulus_metrics(M, precision):
    spec = W.make_annulus(7, 40, 3, seed=3, precision=precision, name="annulus")
    _run_and_compare(M, spec, [0.37 * spec.l_par, 11.5 * spec.l_par], seed=3, noise=1e-3)


@pytest.mark.parametrize("n_par", [1, 2, 3])
def test_tiny_periodic_rows(M, n_par):
    spec = W.make_plane(3, n_par, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP64,
                        name="tiny")
    _run_and_compare(M, spec, [0.0, 0.5 * spec.l_par, 7.25 * spec.l_par, -0.1 * spec.l_par],
                     seed=5, noise=1e-3)


def test_huge_displacement_via_ns_entry(M):
    import torch
    spec = W.make_plane(3, 16, 2, physics=W.EULER, riemann=W.ROE, precision=W.FP64, name="huge")
    op = M.MortarOperator([spec])
    try:
        inp = W.make_inputs(spec, seed=2, noise=1e-3)
        din, oin = H.device_inputs(spec, inp), H.oracle_inputs(spec, inp)
        n, s = (1 << 53) + 5, 0.625
        op.update_ns([n], [s])
        outs = H.gpu_flux(op, [spec], [din])
        ref = H.oracle_flux(spec, oin, n, s)
        err = H.rel_err(spec, (outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy()), ref)
        assert np.max(err) <= 1e-12
        with pytest.raises(M.MortarError):
            op.update_ns([0], [1.0])
        torch.cuda.synchronize()
    finally:
        op.close()


def test_errors_and_determinism(M):
    import torch
    spec = W.make_plane(5, 40, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32)
    op = M.MortarOperator([spec])
    try:
        inp = W.make_inputs(spec, seed=9, noise=1e-3)
        din = H.device_inputs(spec, inp)
        with pytest.raises(M.MortarError, match="no displacement"):
            H.gpu_flux(op, [spec], [din])
        with pytest.raises(M.MortarError, match="invalid"):
            op.update([float("nan")])
        with pytest.raises(M.MortarError, match="invalid"):
            op.update([float("inf")])
        op.update([0.77 * spec.l_par])
        a = H.gpu_flux(op, [spec], [din])
        b = H.gpu_flux(op, [spec], [din])
        for x, y in zip(a[0], b[0]):
            assert torch.equal(x, y)
        with pytest.raises(M.MortarError, match="invalid"):
            op.flux([din["Us"]], [din["Um"]], None, None, [a[0][0]], [a[0][1]])
    finally:
        op.close()


def test_projection_matrices_against_oracle(M):
    for N, ns in ((3, W.GAUSS), (5, W.GAUSS), (4, W.LGL), (9, W.LGL)):
        spec = W.make_plane(N, 8, 1, node_set=ns, precision=W.FP64)
        op = M.MortarOperator([spec])
        try:
            for s in (0.0, 1e-7, 0.3, 0.999):
                op.update_ns([2], [s])
                Pf, Pb = op.projection(0)
                ref = O.projection_matrices(N, ns, s)
                assert np.max(np.abs(Pf - ref["Pf"])) < 1e-13
                assert np.max(np.abs(Pb - ref["Pb"])) < 1e-13
        finally:
            op.close()


@pytest.mark.parametrize("precision", [W.FP64, W.FP32])
def test_conservation_on_device(M, precision):
    spec = W.make_plane(5, 70, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=precision,
                        scramble_seed=4, extra_cols=2)
    op = M.MortarOperator([spec])
    try:
        inp = W.make_inputs(spec, seed=4, noise=1e-2)
        din, oin = H.device_inputs(spec, inp), H.oracle_inputs(spec, inp)
        op.update([2.345 * spec.l_par])
        outs = H.gpu_flux(op, [spec], [din])
        c = op.conservation([outs[0][0]], [outs[0][1]])[0]
        if precision == W.FP64:
            assert np.all(np.abs(c[:, 0] - c[:, 1]) <= 1e-13 * c[:, 2])
        else:
            assert np.all(np.abs(c[:, 0] - c[:, 1]) <= 1e-6 * c[:, 2])
        # the device sums agree with the oracle's sums of the same arrays
        co = O.conservation(spec, outs[0][0].double().cpu().numpy(), outs[0][1].double().cpu().numpy())
        assert np.max(np.abs(c - co)) <= 1e-14 * np.max(np.abs(co))
        # the asynchronous per-stage form writes the same sums into a device array
        import torch
        dev = torch.full((1, 5, 3), float("nan"), dtype=torch.float64, device="cuda:0")
        op.conservation_device([outs[0][0]], [outs[0][1]], dev)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy()[0], c)
    finally:
        op.close()


@pytest.mark.parametrize("N,node_set,physics,riemann,annulus", [
    (1, W.GAUSS, W.EULER, W.ROE, False), (2, W.LGL, W.NS, W.ROE, False),
    (3, W.LGL, W.EULER, W.LF, True), (4, W.GAUSS, W.NS, W.LF, False),
    (5, W.GAUSS, W.NS, W.ROE, True), (6, W.GAUSS, W.EULER, W.ROE, False),
    (7, W.LGL, W.NS, W.ROE, True), (8, W.GAUSS, W.EULER, W.LF, True),
    (9, W.GAUSS, W.EULER, W.ROE, False)])
def test_hybrid_kernel_degrees(M, N, node_set, physics, riemann, annulus):
    """The matrix-core-projection kernel (FP32) over degrees, node sets, fluxes and
    per-point metrics: 37 faces per row (several tiles of 16-face chunks and a ragged
    last one), scrambled columns, two tile lengths."""
    if annulus:
        spec = W.make_annulus(N, 37, 2, seed=N, physics=physics, riemann=riemann,
                              node_set=node_set, mu=1e-3 if physics == W.NS else 0.0,
                              precision=W.FP32, name="hyb-annulus")
    else:
        spec = W.make_plane(N, 37, 2, physics=physics, riemann=riemann, node_set=node_set,
                            mu=1e-3 if physics == W.NS else 0.0, precision=W.FP32,
                            scramble_seed=N, extra_cols=2, name="hyb")
    for tile in (0, 7):
        _run_and_compare(M, spec, [0.41 * spec.l_par, 9.73 * spec.l_par], seed=N, noise=1e-3,
                         check_maps=False, variant=M.KERNEL_HYBRID, tile=tile)


def test_hybrid_kernel_refuses_untileable(M):
    """Degree 9 with Navier-Stokes gradients does not fit the hybrid kernel's LDS tile."""
    spec = W.make_plane(9, 8, 1, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32)
    op = M.MortarOperator([spec])
    try:
        assert M.mortar_set_tuning(op.h, 0, M.KERNEL_HYBRID, 0, 0) == -1
    finally:
        op.close()


@pytest.mark.parametrize("precision,variant",
                         [(p, v) for p in (W.FP32, W.FP64) for v in _VARIANTS[p]])
def test_plane_workload_full_size_all_rows(M, precision, variant):
    """The plane N=5, 128x64, NS Roe+BR1 interface at full size, in every launch variant;
    every row against the oracle (tiles at every XCD boundary of the persistent schedule
    included)."""
    specs, disp = W.config(2, precision=precision)
    spec = specs[0]
    for k in (1, 137):
        _run_and_compare(M, spec, [disp(k)[0]], seed=2, noise=1e-4, check_maps=(k == 137),
                         variant=variant)


@pytest.mark.parametrize("precision,variant",
                         [(p, v) for p in (W.FP32, W.FP64) for v in _VARIANTS[p]])
def test_annulus_workload_full_size_all_rows(M, precision, variant):
    """The annular interface N=7, 512x64 with per-point metrics at full size, every row."""
    specs, disp = W.config(3, precision=precision)
    spec = specs[0]
    _run_and_compare(M, spec, [disp(211)[0]], seed=3, noise=1e-4, check_maps=False,
                     variant=variant)


@pytest.mark.parametrize("variant", _VARIANTS[W.FP32])
def test_euler_n9_workload_full_size_all_rows(M, variant):
    """The plane N=9, 256x256 Euler Roe interface in FP32 (the reference the bf16/fp16
    projection modes are measured against) at full size in every FP32 launch variant,
    including the wide-tile VALU kernel at its longest tile; every row."""
    specs, disp = W.config(5, precision=W.FP32)
    spec = specs[0]
    _run_and_compare(M, spec, [disp(93)[0]], seed=5, noise=1e-4, check_maps=False,
                     variant=variant)


@pytest.mark.parametrize("variant", (0, 2))
def test_turbine_batch_full_size_all_rows(M, variant):
    """The three-interface turbine-like batch at full size in one persistent launch
    (VALU or register-direct batch kernel), every row of every interface."""
    specs, disp = W.config(4, precision=W.FP32)
    d = disp(57)
    op = M.MortarOperator(specs)
    try:
        assert M.mortar_set_tuning(op.h, 0, variant, 0, 0) == 0
        inps = [W.make_inputs(s, seed=4 + i, delta=d[i], noise=1e-4) for i, s in enumerate(specs)]
        dins = [H.device_inputs(s, x) for s, x in zip(specs, inps)]
        op.update(d)
        outs = H.gpu_flux(op, specs, dins)
        for i, s in enumerate(specs):
            n, sf = O.decompose(d[i], s.l_par)
            ref = H.oracle_flux(s, H.oracle_inputs(s, inps[i]), n, sf)
            err = H.rel_err(s, (outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy()), ref)
            print(f"[parity] batch {s.name} variant {variant}: {err}", flush=True)
            assert np.max(err) <= H.TOL[W.FP32], (s.name, err)
    finally:
        op.close()


@pytest.mark.parametrize("precision,variant,tile,grid,n_par,physics", [
    (W.FP32, 0, 0, 0, 70, W.NS), (W.FP32, 3, 0, 0, 70, W.NS), (W.FP32, 0, 7, 8, 70, W.NS),
    (W.FP64, 0, 0, 0, 70, W.NS), (W.FP32, 0, 0, 0, 3, W.NS), (W.FP32, 2, 0, 0, 70, W.NS),
    (W.FP32, 4, 0, 0, 70, W.NS), (W.FP64, 2, 0, 0, 70, W.NS), (W.FP32, 2, 0, 0, 70, W.EULER),
    (W.FP32, 2, 0, 8, 3, W.EULER), (W.BF16_MFMA, 2, 0, 0, 70, W.EULER),
    (W.FP16_MFMA, 2, 0, 0, 70, W.NS)])
def test_fused_conservation_sums(M, precision, variant, tile, grid, n_par, physics):
    """The VALU kernels and the register-direct kernels with 4-byte data write
    per-workgroup conservation partials with their fluxes; the sums taken from them (same
    output arrays) agree with a pass over copies of the arrays to FP64 rounding, on the
    device and on the host alike, also with workgroups that get no tile (3 faces per row)
    and with the kernels that write none (a pass in both cases)."""
    import torch
    spec = W.make_plane(5, n_par, 3, physics=physics, riemann=W.ROE,
                        mu=1e-3 if physics == W.NS else 0.0, precision=precision,
                        scramble_seed=4, extra_cols=2)
    op = M.MortarOperator([spec])
    try:
        assert M.mortar_set_tuning(op.h, 0, variant, tile, grid) == 0
        inp = W.make_inputs(spec, seed=6, noise=1e-2)
        din = H.device_inputs(spec, inp)
        op.update([1.37 * spec.l_par])
        outs = H.gpu_flux(op, [spec], [din], outs=[H.alloc_outputs(spec, fill=0.0)])
        fused = op.conservation([outs[0][0]], [outs[0][1]])[0]
        dev = torch.zeros((1, 5, 3), dtype=torch.float64, device="cuda:0")
        op.conservation_device([outs[0][0]], [outs[0][1]], dev)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy()[0], fused)
        copies = (outs[0][0].clone(), outs[0][1].clone())
        passed = op.conservation([copies[0]], [copies[1]])[0]
        print(f"[parity] conservation variant {variant} precision {precision} physics {physics}: "
              f"fused {fused[:, :2].ravel()[:4]} "
              f"pass {passed[:, :2].ravel()[:4]}", flush=True)
        assert np.all(np.abs(fused - passed) <= 1e-13 * passed[:, 2:3] + 1e-300), (fused, passed)
        # the static and moving integrals agree to the storage rounding of the fluxes
        tol = 1e-13 if precision == W.FP64 else 2e-6
        assert np.all(np.abs(fused[:, 0] - fused[:, 1]) <= tol * fused[:, 2])
    finally:
        op.close()


@pytest.mark.parametrize("precision", [W.FP32, W.BF16_MFMA])
def test_register_direct_schedule_any_grid(M, precision):
    """The register-direct Navier-Stokes launch with 4-byte data runs its waves in rounds
    of consecutive tiles (two groups out of phase, one barrier per round and wave).  Its
    fluxes do not depend on the grid, bit for bit: one workgroup per XCD (several rounds,
    a last round with waves that have no tile), XCDs with different numbers of
    workgroups, more waves than tiles, workgroups with no tile at all.  The conservation
    sums from each launch's fused partials agree with a pass over the arrays to FP64
    rounding, and the fluxes with the oracle."""
    import torch
    spec = W.make_annulus(7, 64, 5, seed=17, precision=precision, name="annulus N=7 64x5")
    inp = W.make_inputs(spec, seed=8, noise=1e-3)
    din, oin = H.device_inputs(spec, inp), H.oracle_inputs(spec, inp)
    d = 2.37 * spec.l_par
    op = M.MortarOperator([spec])
    try:
        op.update([d])
        first = None
        for grid in (8, 13, 40, 0, 520):
            print(f"[parity] register-direct schedule grid {grid} precision {precision}", flush=True)
            assert M.mortar_set_tuning(op.h, 0, M.KERNEL_REGISTER, 0, grid) == 0
            out = H.gpu_flux(op, [spec], [din], outs=[H.alloc_outputs(spec, fill=0.0)])[0]
            fused = op.conservation([out[0]], [out[1]])[0]
            passed = op.conservation([out[0].clone()], [out[1].clone()])[0]
            assert np.all(np.abs(fused - passed) <= 1e-13 * passed[:, 2:3] + 1e-300), (grid, fused, passed)
            if first is None:
                first = out
                n, sf = O.decompose(d, spec.l_par)
                ref = H.oracle_flux(spec, oin, n, sf)
                err = H.rel_err(spec, (out[0].cpu().numpy(), out[1].cpu().numpy()), ref)
                if precision == W.FP32:
                    assert np.max(err) <= H.TOL[W.FP32], err
                else:
                    assert np.max(err) <= 0.1, err      # bf16 operands: see test_gpu_lowprec
            else:
                assert torch.equal(out[0], first[0]) and torch.equal(out[1], first[1]), grid
    finally:
        op.close()


def test_register_direct_batch_schedule_any_grid(M):
    """The same for the batch kernel over the turbine-like degrees (N = 7, 5, 3)."""
    import torch
    specs = [W.make_annulus(7, 48, 4, seed=31, precision=W.FP32, name="a7"),
             W.make_annulus(5, 40, 3, seed=32, precision=W.FP32, name="a5"),
             W.make_plane(3, 33, 3, physics=W.NS, riemann=W.ROE, mu=1e-4, precision=W.FP32,
                          scramble_seed=5, extra_cols=1, name="p3")]
    inps = [W.make_inputs(s, seed=40 + i, noise=1e-3) for i, s in enumerate(specs)]
    dins = [H.device_inputs(s, x) for s, x in zip(specs, inps)]
    disp = [(0.7 + 1.9 * i) * s.l_par for i, s in enumerate(specs)]
    op = M.MortarOperator(specs)
    try:
        op.update(disp)
        first = None
        for grid in (8, 11, 24, 0, 600):
            print(f"[parity] register-direct batch schedule grid {grid}", flush=True)
            assert M.mortar_set_tuning(op.h, 0, M.KERNEL_REGISTER, 0, grid) == 0
            outs = H.gpu_flux(op, specs, dins, outs=[H.alloc_outputs(s, fill=0.0) for s in specs])
            fused = op.conservation([o[0] for o in outs], [o[1] for o in outs])
            passed = op.conservation([o[0].clone() for o in outs], [o[1].clone() for o in outs])
            for i in range(len(specs)):
                assert np.all(np.abs(fused[i] - passed[i]) <= 1e-13 * passed[i][:, 2:3] + 1e-300), (grid, i)
            if first is None:
                first = outs
                for i, s in enumerate(specs):
                    n, sf = O.decompose(disp[i], s.l_par)
                    ref = H.oracle_flux(s, H.oracle_inputs(s, inps[i]), n, sf)
                    err = H.rel_err(s, (outs[i][0].cpu().numpy(), outs[i][1].cpu().numpy()), ref)
                    assert np.max(err) <= H.TOL[W.FP32], (s.name, err)
            else:
                for i in range(len(specs)):
                    assert torch.equal(outs[i][0], first[i][0]) and torch.equal(outs[i][1], first[i][1]), (grid, i)
    finally:
        op.close()


@pytest.mark.parametrize("variant", [0, 2])
def test_prepared_stage_equals_separate_calls(M, variant):
    """MortarStage (arguments marshalled once) gives bitwise the fluxes and conservation
    sums of the separate update / flux / conservation_device calls, stage after stage."""
    import torch
    spec = W.make_plane(5, 37, 3, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32,
                        scramble_seed=2, extra_cols=1)
    din = H.device_inputs(spec, W.make_inputs(spec, seed=4, noise=1e-3))
    op = M.MortarOperator([spec])
    try:
        assert M.mortar_set_tuning(op.h, 0, variant, 0, 0) == 0
        a, b = H.alloc_outputs(spec, fill=0.0), H.alloc_outputs(spec, fill=0.0)
        ca = torch.zeros((1, 5, 3), dtype=torch.float64, device="cuda:0")
        cb = torch.zeros((1, 5, 3), dtype=torch.float64, device="cuda:0")
        stage = op.stage([din["Us"]], [din["Um"]], [din["Gs"]], [din["Gm"]], [a[0]], [a[1]],
                         cons_out=ca)
        for k in range(4):
            d = (0.3 + 5.1 * k) * spec.l_par
            print(f"[parity] prepared stage {k} variant {variant}", flush=True)
            stage([d])
            op.update([d])
            op.flux([din["Us"]], [din["Um"]], [din["Gs"]], [din["Gm"]], [b[0]], [b[1]])
            op.conservation_device([b[0]], [b[1]], cb)
            torch.cuda.synchronize()
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
            assert torch.equal(ca, cb)
    finally:
        op.close()


def test_flux_arrays_beyond_2gib(M):
    """Size limits: an interface whose state and flux arrays pass 2 GiB (FP64 Euler, N = 9,
    1024 x 525 faces, 2.0 GiB per array).  The VALU kernels cannot address it, so the
    default launch takes the MFMA-LDS kernel (64-bit offsets); the register-direct kernel
    addresses arrays up to just below 4 GiB and masks lanes with an offset beyond that.
    Both launches agree everywhere (a masked store landing inside the array would show),
    and the first and last two rows match the oracle on a two-row interface cut from the
    same data (rows are independent chains along the slide).  Inputs are seeded on the
    device: a free stream with 1 % uniform perturbations."""
    import torch
    N, n_par, n_perp = 9, 1024, 525
    spec = W.make_plane(N, n_par, n_perp, physics=W.EULER, riemann=W.ROE, precision=W.FP64,
                        name="beyond-2GiB")
    assert 5 * spec.P * spec.n_face_static * 8 >= 2 ** 31
    g = torch.Generator(device="cuda:0").manual_seed(11)
    rho, vn, p = 1.0, 0.3, 0.71
    U0 = torch.tensor([rho, rho * vn, 0.0, 0.0, p / 0.4 + 0.5 * rho * vn * vn],
                      dtype=torch.float64, device="cuda:0")

    def state(nf):
        r = torch.rand((5, spec.P, nf), generator=g, dtype=torch.float64, device="cuda:0")
        return U0[:, None, None] + 1e-2 * (2.0 * r - 1.0)

    Us, Um = state(spec.n_face_static), state(spec.n_face_moving)
    d = 37.3 * spec.l_par
    n, s = O.decompose(d, spec.l_par)
    op = M.MortarOperator([spec])
    try:
        op.update([d])
        outs = {}
        for variant in (None, 2):
            print(f"[parity] beyond 2 GiB variant {variant}", flush=True)
            if variant is not None:
                assert M.mortar_set_tuning(op.h, 0, variant, 0, 0) == 0
            Fs, Fm = H.alloc_outputs(spec)
            op.flux([Us], [Um], [None], [None], [Fs], [Fm])
            torch.cuda.synchronize()
            outs[variant] = (Fs, Fm)
        assert op.tuning()[0]["variant"] == 2
        for k in (0, 1):
            a, b = outs[None][k], outs[2][k]
            assert not torch.isnan(a).any() and not torch.isnan(b).any()
            assert float((a - b).abs().max()) <= 1e-12 * float(a.abs().max())
        sub = W.make_plane(N, n_par, 2, physics=W.EULER, riemann=W.ROE, precision=W.FP64)
        sub.dS = spec.dS
        for r0 in (0, n_perp - 2):
            cs = torch.from_numpy(spec.face_id_static[r0:r0 + 2].ravel().astype(np.int64)).cuda()
            cm = torch.from_numpy(spec.face_id_moving[r0:r0 + 2].ravel().astype(np.int64)).cuda()
            ref = O.mortar_flux(sub, n, s, Us[:, :, cs].cpu().numpy(), Um[:, :, cm].cpu().numpy())
            for variant, (Fs, Fm) in outs.items():
                got = (Fs[:, :, cs].cpu().numpy(), Fm[:, :, cm].cpu().numpy())
                err = H.rel_err(sub, got, ref)
                print(f"[parity] beyond 2 GiB rows {r0}: variant {variant} err {np.max(err):.2e}", flush=True)
                assert np.max(err) <= H.TOL[W.FP64], (r0, variant, err)
    finally:
        op.close()

"""GPU: mortar_conservation_device_noalloc (partials in the library's static device array,
no allocation) against mortar_conservation_device (partials in handle buffers) through
the C ABI: the same sums, bit for bit, on two calls in a row, the second on a smaller
handle; handles beyond the array's size are refused."""
import numpy as np
import pytest

from paper_2008_04356_amd import workloads as W

from . import _parity as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2008_04356_amd import mortar
    return mortar


def _sums(M, specs, seed, disp):
    """Fluxes of a handle, then the device sums of copies of them (so the existing entry
    point takes its pass over the arrays, the same pass the no-allocation one runs) from
    both entry points."""
    import torch
    op = M.MortarOperator(specs)
    try:
        dins = [H.device_inputs(s, W.make_inputs(s, seed=seed + i, delta=disp[i], noise=1e-3))
                for i, s in enumerate(specs)]
        op.update(disp)
        outs = H.gpu_flux(op, specs, dins, outs=[H.alloc_outputs(s, fill=0.0) for s in specs])
        Fs = [o[0].clone() for o in outs]
        Fm = [o[1].clone() for o in outs]
        ptr = lambda ts: M._ptrs([t.data_ptr() for t in ts])  # noqa: E731
        st = torch.cuda.current_stream().cuda_stream
        ref = torch.full((len(specs), 5, 3), float("nan"), dtype=torch.float64, device="cuda:0")
        got = torch.full((len(specs), 5, 3), float("nan"), dtype=torch.float64, device="cuda:0")
        assert M.mortar_conservation_device(op.h, ptr(Fs), ptr(Fm), ref.data_ptr(), st) == M.OK
        assert M.mortar_conservation_device_noalloc(op.h, ptr(Fs), ptr(Fm), got.data_ptr(), st) == M.OK
        torch.cuda.synchronize()
        return ref.cpu().numpy(), got.cpu().numpy()
    finally:
        op.close()


def test_noalloc_sums_equal_handle_sums_two_calls(M):
    big = [W.make_annulus(5, 300, 40, seed=1, precision=W.FP32, name="noalloc-annulus"),
           W.make_plane(3, 64, 32, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32,
                        scramble_seed=2, extra_cols=3, name="noalloc-plane")]
    small = [W.make_plane(4, 9, 2, physics=W.EULER, riemann=W.LF, precision=W.FP64,
                          scramble_seed=5, name="noalloc-small")]
    for specs, seed in ((big, 11), (small, 21)):
        print(f"[noalloc] {[s.name for s in specs]}", flush=True)
        disp = [0.37 * s.l_par for s in specs]
        ref, got = _sums(M, specs, seed, disp)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(ref, got), (ref, got)


def test_noalloc_refuses_more_interfaces_than_its_array(M):
    import torch
    specs = [W.make_plane(2, 4, 1, physics=W.EULER, riemann=W.LF, precision=W.FP64) for _ in range(9)]
    op = M.MortarOperator(specs)
    try:
        F = [torch.zeros((5, s.P, s.n_face_static), dtype=torch.float64, device="cuda:0") for s in specs]
        out = torch.zeros((9, 5, 3), dtype=torch.float64, device="cuda:0")
        p = M._ptrs([t.data_ptr() for t in F])
        rc = M.mortar_conservation_device_noalloc(op.h, p, p, out.data_ptr(),
                                                  torch.cuda.current_stream().cuda_stream)
        assert rc == M.ERR_UNSUPPORTED
    finally:
        op.close()

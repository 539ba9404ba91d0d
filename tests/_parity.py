"""Helpers for the GPU parity tests: run the HIP path through the C ABI binding and the
FP64 oracle on the same seeded inputs, and measure the per-variable relative error.

Error norm per output variable v (both sides together):
    e_v = max|F_gpu - F_ref| / max(max|F_ref_v|, 1e-3 * max_v' max|F_ref_v'|)
For FP32 runs the oracle consumes the FP32-rounded inputs promoted to FP64."""
import numpy as np

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

TOL = {W.FP64: 1e-12, W.FP32: 1e-5}


def torch_dtype(precision):
    import torch
    return torch.float64 if precision == W.FP64 else torch.float32


def to_device(arr, precision, device="cuda:0"):
    import torch
    if arr is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(W.round_to(arr, precision))).to(device)


def device_inputs(spec, inp):
    return {k: to_device(v, spec.precision) for k, v in inp.items()}


def oracle_inputs(spec, inp):
    """What the oracle sees: the device inputs' values in FP64."""
    return {k: (None if v is None else np.asarray(W.round_to(v, spec.precision), dtype=np.float64))
            for k, v in inp.items()}


def alloc_outputs(spec, fill=np.nan):
    import torch
    dt = torch_dtype(spec.precision)
    Fs = torch.full((5, spec.P, spec.n_face_static), fill, dtype=dt, device="cuda:0")
    Fm = torch.full((5, spec.P, spec.n_face_moving), fill, dtype=dt, device="cuda:0")
    return Fs, Fm


def gpu_flux(op, specs, dins, outs=None):
    import torch
    if outs is None:
        outs = [alloc_outputs(s) for s in specs]
    op.flux([d["Us"] for d in dins], [d["Um"] for d in dins],
            [d["Gs"] for d in dins], [d["Gm"] for d in dins],
            [o[0] for o in outs], [o[1] for o in outs])
    torch.cuda.synchronize()
    return outs


def oracle_threads():
    """Threads for the oracle's row ranges: the usable cores, at most 16."""
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_flux(spec, oin, n, s, rows=None):
    return O.mortar_flux(spec, n, s, oin["Us"], oin["Um"], oin["Gs"], oin["Gm"], rows=rows,
                         threads=oracle_threads())


def rel_err(spec, F_gpu, F_ref, rows=None):
    """Per-variable error over the interface's columns (optionally only some rows)."""
    fs = spec.face_id_static
    fm = spec.face_id_moving
    if rows is not None:
        fs, fm = fs[rows[0]:rows[1]], fm[rows[0]:rows[1]]
    cs, cm = fs.ravel(), fm.ravel()
    g = [np.asarray(F_gpu[0], dtype=np.float64)[:, :, cs], np.asarray(F_gpu[1], dtype=np.float64)[:, :, cm]]
    r = [F_ref[0][:, :, cs], F_ref[1][:, :, cm]]
    scale_v = np.array([max(np.max(np.abs(r[0][v])), np.max(np.abs(r[1][v]))) for v in range(5)])
    floor = 1e-3 * np.max(scale_v)
    err = np.zeros(5)
    for v in range(5):
        d = max(np.max(np.abs(g[0][v] - r[0][v])), np.max(np.abs(g[1][v] - r[1][v])))
        err[v] = d / max(scale_v[v], floor)
    return err

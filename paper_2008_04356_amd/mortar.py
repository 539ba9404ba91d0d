"""Thin ctypes binding of libmortar.so (C ABI in include/mortar.h).

Argument marshalling only: every step of the operator runs in the HIP library.  Torch
is used for device memory and streams.  There is no fallback: if the library is missing
or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmortar.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OOM, ERR_HIP, ERR_NOT_READY = 0, -1, -2, -3, -4, -5
GEOM_PLANE, GEOM_ANNULUS = 0, 1
NODES_GAUSS, NODES_LGL = 0, 1
EULER, NAVIER_STOKES = 0, 1
FLUX_LF, FLUX_ROE = 0, 1
FP64, FP32, BF16_MFMA, FP16_MFMA = 0, 1, 2, 3

_ip = C.POINTER(C.c_int32)
_dp = C.POINTER(C.c_double)
_vpp = C.POINTER(C.c_void_p)


class mortar_iface_desc(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32), ("N", C.c_int32), ("node_set", C.c_int32),
        ("n_par", C.c_int32), ("n_perp", C.c_int32),
        ("n_face_static", C.c_int32), ("n_face_moving", C.c_int32),
        ("face_id_static", _ip), ("face_id_moving", _ip),
        ("owner_static", _ip), ("owner_moving", _ip),
        ("l_par", C.c_double), ("normal", C.c_double * 3), ("dS", C.c_double),
        ("metrics", _dp),
        ("physics", C.c_int32), ("riemann", C.c_int32), ("precision", C.c_int32),
        ("reserved", C.c_int32),
        ("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double),
    ]


class mortar_tuning(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tile_len", C.c_int32), ("grid", C.c_int32),
                ("reserved", C.c_int32)]


KERNEL_VALU, KERNEL_MFMA_LDS, KERNEL_REGISTER, KERNEL_VALU_WIDE, KERNEL_HYBRID = 0, 1, 2, 3, 4


class MortarError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2008_04356_amd/build.py "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    L.mortar_validate.argtypes = [C.POINTER(mortar_iface_desc), C.c_int]
    L.mortar_setup.argtypes = [C.POINTER(mortar_iface_desc), C.c_int, C.POINTER(C.c_void_p)]
    L.mortar_update_displacement.argtypes = [C.c_void_p, _dp, C.c_void_p]
    L.mortar_update_displacement_ns.argtypes = [C.c_void_p, C.POINTER(C.c_int64), _dp, C.c_void_p]
    L.mortar_flux.argtypes = [C.c_void_p, _vpp, _vpp, _vpp, _vpp, _vpp, _vpp, C.c_void_p]
    L.mortar_lifting.argtypes = [C.c_void_p, _vpp, _vpp, _vpp, _vpp, C.c_void_p]
    L.mortar_destroy.argtypes = [C.c_void_p]
    L.mortar_error_string.argtypes = [C.c_int]
    L.mortar_error_string.restype = C.c_char_p
    L.mortar_decompose_displacement.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int64), _dp]
    L.mortar_basis.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.mortar_get_displacement.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64), _dp]
    L.mortar_get_index_map.argtypes = [C.c_void_p, C.c_int, C.c_int, _ip, _ip]
    L.mortar_get_projection.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
    L.mortar_get_pairing.argtypes = [C.c_void_p, C.c_int, _ip]
    L.mortar_conservation.argtypes = [C.c_void_p, _vpp, _vpp, _dp, C.c_void_p]
    L.mortar_conservation_device.argtypes = [C.c_void_p, _vpp, _vpp, C.c_void_p, C.c_void_p]
    L.mortar_conservation_device_noalloc.argtypes = [C.c_void_p, _vpp, _vpp, C.c_void_p, C.c_void_p]
    L.mortar_graph_create.argtypes = [C.c_void_p, _vpp, _vpp, _vpp, _vpp, _vpp, _vpp,
                                      C.POINTER(C.c_void_p)]
    L.mortar_graph_create_cons.argtypes = [C.c_void_p, _vpp, _vpp, _vpp, _vpp, _vpp, _vpp,
                                           C.c_void_p, C.POINTER(C.c_void_p)]
    L.mortar_graph_launch.argtypes = [C.c_void_p, _dp, C.c_void_p]
    L.mortar_graph_destroy.argtypes = [C.c_void_p]
    L.mortar_autotune.argtypes = [C.c_void_p, _vpp, _vpp, _vpp, _vpp, _vpp, _vpp, C.c_int,
                                  C.c_void_p]
    L.mortar_get_tuning.argtypes = [C.c_void_p, C.c_int, C.POINTER(mortar_tuning)]
    L.mortar_set_tuning.argtypes = [C.c_void_p, C.c_int, C.POINTER(mortar_tuning)]
    return L


lib = _load()


def _check(rc: int, what: str):
    if rc != OK:
        raise MortarError(f"{what}: {lib.mortar_error_string(rc).decode()} ({rc})")


# ---- same names as the C ABI (argument marshalling only) -----------------------------

def mortar_validate(descs) -> int:
    arr = (mortar_iface_desc * len(descs))(*descs)
    return lib.mortar_validate(arr, len(descs))


def mortar_setup(descs) -> C.c_void_p:
    arr = (mortar_iface_desc * len(descs))(*descs)
    h = C.c_void_p()
    _check(lib.mortar_setup(arr, len(descs), C.byref(h)), "mortar_setup")
    return h


def mortar_update_displacement(h, disp: Sequence[float], stream: int = 0) -> int:
    d = (C.c_double * len(disp))(*[float(x) for x in disp])
    return lib.mortar_update_displacement(h, d, C.c_void_p(stream))


def mortar_update_displacement_ns(h, n: Sequence[int], s: Sequence[float], stream: int = 0) -> int:
    nn = (C.c_int64 * len(n))(*[int(x) for x in n])
    ss = (C.c_double * len(s))(*[float(x) for x in s])
    return lib.mortar_update_displacement_ns(h, nn, ss, C.c_void_p(stream))


def _ptrs(ts):
    if ts is None:
        return None
    return (C.c_void_p * len(ts))(*[None if t is None else C.c_void_p(int(t)) for t in ts])


def mortar_flux(h, Us, Um, Gs, Gm, Fs, Fm, stream: int = 0) -> int:
    """Each argument: a sequence of device addresses (ints) or None entries."""
    return lib.mortar_flux(h, _ptrs(Us), _ptrs(Um), _ptrs(Gs), _ptrs(Gm), _ptrs(Fs), _ptrs(Fm),
                           C.c_void_p(stream))


def mortar_lifting(h, Us, Um, Ls, Lm, stream: int = 0) -> int:
    """Each argument: a sequence of device addresses (ints)."""
    return lib.mortar_lifting(h, _ptrs(Us), _ptrs(Um), _ptrs(Ls), _ptrs(Lm), C.c_void_p(stream))


def mortar_graph_create(h, Us, Um, Gs, Gm, Fs, Fm):
    g = C.c_void_p()
    _check(lib.mortar_graph_create(h, _ptrs(Us), _ptrs(Um), _ptrs(Gs), _ptrs(Gm), _ptrs(Fs),
                                   _ptrs(Fm), C.byref(g)), "mortar_graph_create")
    return g


def mortar_graph_create_cons(h, Us, Um, Gs, Gm, Fs, Fm, d_cons: int):
    g = C.c_void_p()
    _check(lib.mortar_graph_create_cons(h, _ptrs(Us), _ptrs(Um), _ptrs(Gs), _ptrs(Gm), _ptrs(Fs),
                                        _ptrs(Fm), C.c_void_p(d_cons), C.byref(g)),
           "mortar_graph_create_cons")
    return g


def mortar_graph_launch(g, disp: Sequence[float], stream: int = 0) -> int:
    d = (C.c_double * len(disp))(*[float(x) for x in disp])
    return lib.mortar_graph_launch(g, d, C.c_void_p(stream))


def mortar_graph_destroy(g) -> int:
    return lib.mortar_graph_destroy(g)


def mortar_autotune(h, Us, Um, Gs, Gm, Fs, Fm, reps: int = 5, stream: int = 0) -> int:
    return lib.mortar_autotune(h, _ptrs(Us), _ptrs(Um), _ptrs(Gs), _ptrs(Gm), _ptrs(Fs),
                               _ptrs(Fm), int(reps), C.c_void_p(stream))


def mortar_get_tuning(h, iface: int):
    t = mortar_tuning()
    _check(lib.mortar_get_tuning(h, iface, C.byref(t)), "mortar_get_tuning")
    return {"variant": t.variant, "tile_len": t.tile_len, "grid": t.grid}


def mortar_set_tuning(h, iface: int, variant: int, tile_len: int = 0, grid: int = 0) -> int:
    t = mortar_tuning(int(variant), int(tile_len), int(grid), 0)
    return lib.mortar_set_tuning(h, iface, C.byref(t))


def mortar_conservation_device(h, Fs, Fm, d_out: int, stream: int = 0) -> int:
    return lib.mortar_conservation_device(h, Fs, Fm, C.c_void_p(int(d_out)), C.c_void_p(stream))


def mortar_conservation_device_noalloc(h, Fs, Fm, d_out: int, stream: int = 0) -> int:
    return lib.mortar_conservation_device_noalloc(h, Fs, Fm, C.c_void_p(int(d_out)), C.c_void_p(stream))


def mortar_destroy(h) -> int:
    return lib.mortar_destroy(h)


def mortar_error_string(code: int) -> str:
    return lib.mortar_error_string(code).decode()


def mortar_basis(N: int, node_set: int):
    x = np.zeros(N + 1)
    w = np.zeros(N + 1)
    _check(lib.mortar_basis(N, node_set, x.ctypes.data_as(_dp), w.ctypes.data_as(_dp)), "mortar_basis")
    return x, w


def mortar_decompose_displacement(delta: float, l_par: float):
    n = C.c_int64()
    s = C.c_double()
    _check(lib.mortar_decompose_displacement(delta, l_par, C.byref(n), C.byref(s)),
           "mortar_decompose_displacement")
    return int(n.value), float(s.value)


# ---- descriptors from workload specs --------------------------------------------------

class _Keep:
    pass


def make_desc(spec, keep: Optional[list] = None) -> mortar_iface_desc:
    """Descriptor of a workloads.InterfaceSpec (duck-typed).  Host arrays are kept alive
    in `keep` until mortar_setup has copied them."""
    d = mortar_iface_desc()
    k = _Keep()
    k.fs = np.ascontiguousarray(spec.face_id_static, dtype=np.int32).ravel()
    k.fm = np.ascontiguousarray(spec.face_id_moving, dtype=np.int32).ravel()
    d.geometry = int(getattr(spec, "geometry", 0))
    d.N, d.node_set = int(spec.N), int(spec.node_set)
    d.n_par, d.n_perp = int(spec.n_par), int(spec.n_perp)
    d.n_face_static, d.n_face_moving = int(spec.n_face_static), int(spec.n_face_moving)
    d.face_id_static = k.fs.ctypes.data_as(_ip)
    d.face_id_moving = k.fm.ctypes.data_as(_ip)
    for name in ("owner_static", "owner_moving"):
        arr = getattr(spec, name, None)
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.int32).ravel()
            setattr(k, name, a)
            setattr(d, name, a.ctypes.data_as(_ip))
    d.l_par = float(spec.l_par)
    for i in range(3):
        d.normal[i] = float(spec.normal[i])
    d.dS = float(spec.dS)
    if getattr(spec, "metrics", None) is not None:
        k.met = np.ascontiguousarray(spec.metrics, dtype=np.float64)
        d.metrics = k.met.ctypes.data_as(_dp)
    d.physics, d.riemann, d.precision = int(spec.physics), int(spec.riemann), int(spec.precision)
    d.gamma, d.mu, d.Pr = float(spec.gamma), float(spec.mu), float(spec.Pr)
    if keep is not None:
        keep.append(k)
    d._keep = k
    return d


# ---- convenience object (torch tensors in, torch tensors out) ------------------------

def _dtype_of(spec):
    import torch
    return torch.float64 if int(spec.precision) == FP64 else torch.float32


def _check_tensor(t, spec, shape, what):
    """A face array handed to the library: a contiguous CUDA tensor of the interface's
    element type and the exact shape the kernels address (anything else would make them
    read or write outside the allocation)."""
    if t is None:
        raise MortarError(f"invalid argument: {what}: missing tensor")
    if not getattr(t, "is_cuda", False):
        raise MortarError(f"invalid argument: {what}: must be a CUDA tensor")
    if not t.is_contiguous():
        raise MortarError(f"invalid argument: {what}: must be contiguous")
    if t.dtype != _dtype_of(spec):
        raise MortarError(f"invalid argument: {what}: dtype {t.dtype}, the interface needs {_dtype_of(spec)}")
    if tuple(t.shape) != tuple(shape):
        raise MortarError(f"invalid argument: {what}: shape {tuple(t.shape)}, the interface needs {tuple(shape)}")


def _check_list(ts, specs, kind, what):
    """kind: 'state' [5][P][n_face], 'grad' [3][5][P][n_face] (NS only; None for Euler),
    'lift' [3][5][P][n_face]; side 's' or 'm' picks the static or moving column count."""
    if ts is None:
        if kind == "grad" and all(int(s.physics) != NAVIER_STOKES for s in specs):
            return
        raise MortarError(f"invalid argument: {what}: missing")
    if len(ts) != len(specs):
        raise MortarError(f"invalid argument: {what}: {len(ts)} entries for {len(specs)} interfaces")
    side = what[-1]
    for i, (t, sp) in enumerate(zip(ts, specs)):
        nf = sp.n_face_static if side == "s" else sp.n_face_moving
        P = (int(sp.N) + 1) ** 2
        if kind == "grad":
            if int(sp.physics) != NAVIER_STOKES:
                continue
            shape = (3, 5, P, nf)
        elif kind == "lift":
            shape = (3, 5, P, nf)
        else:
            shape = (5, P, nf)
        _check_tensor(t, sp, shape, f"{what}[{i}]")


def _check_disp(disp, specs, what):
    if len(disp) != len(specs):
        raise MortarError(f"invalid argument: {what}: {len(disp)} displacements for {len(specs)} interfaces")


def _check_flux_args(specs, Us, Um, Gs, Gm, Fs, Fm):
    _check_list(Us, specs, "state", "U_s")
    _check_list(Um, specs, "state", "U_m")
    _check_list(Gs, specs, "grad", "G_s")
    _check_list(Gm, specs, "grad", "G_m")
    _check_list(Fs, specs, "state", "F_s")
    _check_list(Fm, specs, "state", "F_m")


class MortarOperator:
    """Owns a library handle for a list of interfaces."""

    def __init__(self, specs):
        self.specs = list(specs)
        keep = []
        self.descs = [make_desc(s, keep) for s in self.specs]
        self.h = mortar_setup(self.descs)
        del keep

    def close(self):
        if self.h:
            _check(mortar_destroy(self.h), "mortar_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream(stream):
        if stream is None:
            import torch
            return torch.cuda.current_stream().cuda_stream
        return int(stream)

    def update(self, disp, stream=None):
        _check_disp(disp, self.specs, "mortar_update_displacement")
        _check(mortar_update_displacement(self.h, disp, self._stream(stream)),
               "mortar_update_displacement")

    def update_ns(self, n, s, stream=None):
        _check_disp(n, self.specs, "mortar_update_displacement_ns")
        _check_disp(s, self.specs, "mortar_update_displacement_ns")
        _check(mortar_update_displacement_ns(self.h, n, s, self._stream(stream)),
               "mortar_update_displacement_ns")

    def flux(self, Us, Um, Gs, Gm, Fs, Fm, stream=None):
        _check_flux_args(self.specs, Us, Um, Gs, Gm, Fs, Fm)
        p = lambda ts: None if ts is None else [None if t is None else t.data_ptr() for t in ts]  # noqa: E731
        _check(mortar_flux(self.h, p(Us), p(Um), p(Gs), p(Gm), p(Fs), p(Fm), self._stream(stream)),
               "mortar_flux")

    def stage(self, Us, Um, Gs, Gm, Fs, Fm, cons_out=None, stream=None):
        """One stage for fixed face buffers with the arguments marshalled once (see
        MortarStage): stage(disp) runs the displacement update, the flux and, with cons_out,
        the device conservation sums."""
        return MortarStage(self, Us, Um, Gs, Gm, Fs, Fm, cons_out, stream)

    def lifting(self, Us, Um, Ls, Lm, stream=None):
        """BR1 lifting surface term: Ls[i], Lm[i] [3][5][P][n_face] tensors (written)."""
        _check_list(Us, self.specs, "state", "U_s")
        _check_list(Um, self.specs, "state", "U_m")
        _check_list(Ls, self.specs, "lift", "L_s")
        _check_list(Lm, self.specs, "lift", "L_m")
        p = lambda ts: [t.data_ptr() for t in ts]  # noqa: E731
        _check(mortar_lifting(self.h, p(Us), p(Um), p(Ls), p(Lm), self._stream(stream)), "mortar_lifting")

    def tuning_key(self):
        """What a tuning depends on: the device, and every interface's shape and mode."""
        import torch
        dev = torch.cuda.get_device_properties(torch.cuda.current_device())
        arch = getattr(dev, "gcnArchName", dev.name)
        parts = [f"{s.N}/{s.node_set}/{s.n_par}x{s.n_perp}/{s.n_face_static},{s.n_face_moving}/"
                 f"{s.physics}/{s.riemann}/{s.precision}/{int(s.metrics is not None)}"
                 for s in self.specs]
        return arch + "|" + ";".join(parts)

    def tuning(self):
        return [mortar_get_tuning(self.h, i) for i in range(len(self.specs))]

    def set_tuning(self, tunings):
        for i, t in enumerate(tunings):
            _check(mortar_set_tuning(self.h, i, t["variant"], t["tile_len"], t["grid"]),
                   "mortar_set_tuning")

    def autotune(self, Us, Um, Gs, Gm, Fs, Fm, reps=5, cache=None, stream=None):
        """Picks the launch of every interface by timing the candidates on these buffers
        (outputs are overwritten).  cache: path of a JSON file mapping tuning_key() to the
        chosen tunings; a hit applies the stored choice without timing."""
        import json
        import os
        key = self.tuning_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
            if key in table:
                self.set_tuning(table[key])
                return table[key]
        _check_flux_args(self.specs, Us, Um, Gs, Gm, Fs, Fm)
        p = lambda ts: None if ts is None else [None if t is None else t.data_ptr() for t in ts]  # noqa: E731
        _check(mortar_autotune(self.h, p(Us), p(Um), p(Gs), p(Gm), p(Fs), p(Fm), reps,
                               self._stream(stream)), "mortar_autotune")
        chosen = self.tuning()
        if cache:
            table[key] = chosen
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return chosen

    def displacement(self, iface=0):
        n = C.c_int64()
        s = C.c_double()
        _check(lib.mortar_get_displacement(self.h, iface, C.byref(n), C.byref(s)),
               "mortar_get_displacement")
        return int(n.value), float(s.value)

    def index_map(self, iface=0, side=0):
        sp = self.specs[iface]
        F = sp.n_par * sp.n_perp
        nf = sp.n_face_static if side == 0 else sp.n_face_moving
        A = np.zeros((5, 2 * F), dtype=np.int32)
        m = np.zeros((2, nf), dtype=np.int32)
        _check(lib.mortar_get_index_map(self.h, iface, side, A.ctypes.data_as(_ip),
                                        m.ctypes.data_as(_ip)), "mortar_get_index_map")
        return A, m

    def pairing(self, iface=0):
        """[2][n_par] int32: moving face index of mortar (i_par, i_sub) in every row."""
        pair = np.zeros((2, self.specs[iface].n_par), dtype=np.int32)
        _check(lib.mortar_get_pairing(self.h, iface, pair.ctypes.data_as(_ip)), "mortar_get_pairing")
        return pair

    def projection(self, iface=0):
        NP = self.specs[iface].N + 1
        Pf = np.zeros((4, NP, NP))
        Pb = np.zeros((4, NP, NP))
        _check(lib.mortar_get_projection(self.h, iface, Pf.ctypes.data_as(_dp),
                                         Pb.ctypes.data_as(_dp)), "mortar_get_projection")
        return Pf, Pb

    def graph(self, Us, Um, Gs, Gm, Fs, Fm, cons_out=None):
        """Captures one stage for these fixed buffers; see MortarGraph.  cons_out (a
        contiguous CUDA float64 tensor [n_iface][5][3]) puts the stage's conservation
        sums into the same graph."""
        return MortarGraph(self, Us, Um, Gs, Gm, Fs, Fm, cons_out)

    def _check_cons(self, Fs, Fm, out=None):
        import torch
        _check_list(Fs, self.specs, "state", "F_s")
        _check_list(Fm, self.specs, "state", "F_m")
        if out is not None:
            if not (getattr(out, "is_cuda", False) and out.is_contiguous() and out.dtype == torch.float64
                    and tuple(out.shape) == (len(self.specs), 5, 3)):
                raise MortarError(f"invalid argument: conservation output: needs a contiguous CUDA float64 tensor "
                                  f"of shape ({len(self.specs)}, 5, 3)")

    def conservation_device(self, Fs, Fm, out, stream=None):
        """Asynchronous sums into the device tensor out (float64, [n_iface, 5, 3])."""
        self._check_cons(Fs, Fm, out)
        p = lambda ts: _ptrs([t.data_ptr() for t in ts])  # noqa: E731
        _check(mortar_conservation_device(self.h, p(Fs), p(Fm), out.data_ptr(),
                                          self._stream(stream)), "mortar_conservation_device")

    def conservation_device_noalloc(self, Fs, Fm, out, stream=None):
        """The same sums with the library's static partials array (no allocation)."""
        self._check_cons(Fs, Fm, out)
        p = lambda ts: _ptrs([t.data_ptr() for t in ts])  # noqa: E731
        _check(mortar_conservation_device_noalloc(self.h, p(Fs), p(Fm), out.data_ptr(),
                                                  self._stream(stream)),
               "mortar_conservation_device_noalloc")

    def conservation(self, Fs, Fm, stream=None):
        self._check_cons(Fs, Fm)
        out = np.zeros((len(self.specs), 5, 3))
        p = lambda ts: _ptrs([t.data_ptr() for t in ts])  # noqa: E731
        _check(lib.mortar_conservation(self.h, p(Fs), p(Fm), out.ctypes.data_as(_dp),
                                       C.c_void_p(self._stream(stream))), "mortar_conservation")
        return out


class MortarStage:
    """A stage launcher for fixed face buffers: the pointer arrays, the stream and the
    displacement array are built once, so a call costs three C calls
    (mortar_update_displacement, mortar_flux, and mortar_conservation_device into cons_out,
    a float64 device tensor [n_iface, 5, 3], when given).  The stream is the one given, else
    the current stream at construction."""

    def __init__(self, op, Us, Um, Gs, Gm, Fs, Fm, cons_out=None, stream=None):
        _check_flux_args(op.specs, Us, Um, Gs, Gm, Fs, Fm)
        if cons_out is not None:
            op._check_cons(Fs, Fm, cons_out)
        p = lambda ts: None if ts is None else _ptrs([None if t is None else t.data_ptr() for t in ts])  # noqa: E731
        self._keep = (op, Us, Um, Gs, Gm, Fs, Fm, cons_out)
        self._n = len(op.specs)
        self._h = op.h
        self._args = (p(Us), p(Um), p(Gs), p(Gm), p(Fs), p(Fm))
        self._st = C.c_void_p(op._stream(stream))
        self._disp = (C.c_double * len(op.specs))()
        self._cons = None if cons_out is None else \
            (self._args[4], self._args[5], C.c_void_p(cons_out.data_ptr()))

    def __call__(self, disp):
        if len(disp) != self._n:
            raise MortarError(f"invalid argument: mortar stage: {len(disp)} displacements for {self._n} interfaces")
        d = self._disp
        for i, x in enumerate(disp):
            d[i] = x
        rc = lib.mortar_update_displacement(self._h, d, self._st)
        if rc == OK:
            rc = lib.mortar_flux(self._h, *self._args, self._st)
        if rc == OK and self._cons is not None:
            rc = lib.mortar_conservation_device(self._h, *self._cons, self._st)
        _check(rc, "mortar stage")


class MortarGraph:
    """One stage of an operator captured as a HIP graph for fixed face buffers; each
    launch(disp) updates the displacement and replays the graph (with cons_out, the
    graph also writes the stage's conservation sums there)."""

    def __init__(self, op, Us, Um, Gs, Gm, Fs, Fm, cons_out=None):
        _check_flux_args(op.specs, Us, Um, Gs, Gm, Fs, Fm)
        p = lambda ts: None if ts is None else [None if t is None else t.data_ptr() for t in ts]  # noqa: E731
        self.op = op
        self._keep = (Us, Um, Gs, Gm, Fs, Fm, cons_out)
        self.g = None
        if cons_out is None:
            self.g = mortar_graph_create(op.h, p(Us), p(Um), p(Gs), p(Gm), p(Fs), p(Fm))
        else:
            op._check_cons(Fs, Fm, cons_out)
            self.g = mortar_graph_create_cons(op.h, p(Us), p(Um), p(Gs), p(Gm), p(Fs), p(Fm),
                                              cons_out.data_ptr())

    def launch(self, disp, stream=None):
        _check_disp(disp, self.op.specs, "mortar_graph_launch")
        _check(mortar_graph_launch(self.g, disp, MortarOperator._stream(stream)),
               "mortar_graph_launch")

    def close(self):
        if self.g:
            _check(mortar_graph_destroy(self.g), "mortar_graph_destroy")
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes front end of the plain FP64 CPU oracle (oracle/mortar_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline
leg of the benchmark.  The product library never imports it, and it imports nothing
from the product package.

Interface descriptions are duck-typed: any object with the attributes N, node_set,
n_par, n_perp, face_id_static, face_id_moving, n_face_static, n_face_moving, physics,
riemann, gamma, mu, Pr, normal, dS and metrics (None or a [4][P][n_face_static] array).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

GAUSS, LGL = 0, 1
EULER, NS = 0, 1
LF, ROE, ROE_NOFIX, AVG, LIFT = 0, 1, 2, 99, 100

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Iface(C.Structure):
    _fields_ = [
        ("N", C.c_int), ("node_set", C.c_int), ("n_par", C.c_int), ("n_perp", C.c_int),
        ("face_id_static", _ip), ("face_id_moving", _ip),
        ("n_face_static", C.c_int), ("n_face_moving", C.c_int),
        ("physics", C.c_int), ("riemann", C.c_int),
        ("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double),
        ("normal", C.c_double * 3), ("dS", C.c_double), ("metrics", _dp),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            import importlib.util
            spec = importlib.util.spec_from_file_location("_oracle_build", os.path.join(HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        _lib = C.CDLL(LIB_PATH)
        L = _lib
        L.orc_nodes.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.orc_gauss_rule.argtypes = [C.c_int, _dp, _dp]
        L.orc_lagrange.argtypes = [C.c_int, _dp, C.c_int, C.c_double]
        L.orc_lagrange.restype = C.c_double
        L.orc_decompose.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int64), _dp]
        L.orc_pair_bruteforce.argtypes = [C.c_int, C.c_int64, C.c_double, C.c_int, C.c_int]
        L.orc_pair_relation.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_int]
        L.orc_projection_matrices.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.orc_point_flux.argtypes = [_dp, _dp, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int,
                                     C.c_double, C.c_double, C.c_double, _dp]
        L.orc_euler_normal_flux.argtypes = [_dp, _dp, C.c_double, _dp]
        L.orc_viscous_normal_flux.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
        L.orc_mortar_flux.argtypes = [C.POINTER(_Iface), C.c_int64, C.c_double,
                                      _dp, _dp, _dp, _dp, _dp, _dp, C.c_int, C.c_int]
        L.orc_sort_mortars.argtypes = [C.c_int, _ip, _ip, _ip, C.c_int, C.c_int]
        L.orc_index_map.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, _ip, C.c_int, _ip, _ip, _ip]
        L.orc_conservation.argtypes = [C.POINTER(_Iface), _dp, _dp, _dp]
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def nodes(N: int, node_set: int = GAUSS):
    x = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if lib().orc_nodes(N, node_set, _d(x), _d(w)):
        raise ValueError("bad node set request")
    return x, w


def gauss_rule(q: int):
    x = np.zeros(q)
    w = np.zeros(q)
    if lib().orc_gauss_rule(q, _d(x), _d(w)):
        raise ValueError("bad rule size")
    return x, w


def lagrange(N: int, x, j: int, xi: float) -> float:
    x = _f64(x)
    return lib().orc_lagrange(N, _d(x), j, xi)


def decompose(delta: float, l_par: float):
    n = C.c_int64()
    s = C.c_double()
    lib().orc_decompose(delta, l_par, C.byref(n), C.byref(s))
    return int(n.value), float(s.value)


def pair_bruteforce(n_par: int, n: int, s: float, i_par: int, i_sub: int) -> int:
    return lib().orc_pair_bruteforce(n_par, n, s, i_par, i_sub)


def pair_relation(n_par: int, n: int, i_par: int, i_sub: int) -> int:
    return lib().orc_pair_relation(n_par, n, i_par, i_sub)


def projection_matrices(N: int, node_set: int, s: float):
    NP = N + 1
    M = np.zeros((NP, NP))
    S = np.zeros((4, NP, NP))
    Pf = np.zeros((4, NP, NP))
    Pb = np.zeros((4, NP, NP))
    J = np.zeros(4)
    rc = lib().orc_projection_matrices(N, node_set, s, _d(M), _d(S), _d(Pf), _d(Pb), _d(J))
    if rc:
        raise ValueError(f"projection matrices failed ({rc})")
    return {"M": M, "S": S, "Pf": Pf, "Pb": Pb, "J": J}


def point_flux(UL, UR, gL=None, gR=None, normal=(1.0, 0.0, 0.0), dS=1.0, physics=EULER,
               riemann=ROE, gamma=1.4, mu=0.0, Pr=0.72):
    UL, UR = _f64(UL), _f64(UR)
    gL = _f64(np.zeros(15) if gL is None else gL)
    gR = _f64(np.zeros(15) if gR is None else gR)
    n = _f64(normal)
    F = np.zeros(5)
    lib().orc_point_flux(_d(UL), _d(UR), _d(gL), _d(gR), _d(n), dS, physics, riemann,
                         gamma, mu, Pr, _d(F))
    return F


def euler_normal_flux(U, normal, gamma=1.4):
    U, n = _f64(U), _f64(normal)
    F = np.zeros(5)
    lib().orc_euler_normal_flux(_d(U), _d(n), gamma, _d(F))
    return F


def viscous_normal_flux(U, g, normal, gamma=1.4, mu=1e-4, Pr=0.72):
    U, g, n = _f64(U), _f64(g), _f64(normal)
    F = np.zeros(5)
    lib().orc_viscous_normal_flux(_d(U), _d(g), _d(n), gamma, mu, Pr, _d(F))
    return F


class _Keep:
    """Holds numpy buffers alive while a C struct points at them."""


def _iface(spec):
    keep = _Keep()
    keep.fs = np.ascontiguousarray(spec.face_id_static, dtype=np.int32).ravel()
    keep.fm = np.ascontiguousarray(spec.face_id_moving, dtype=np.int32).ravel()
    st = _Iface()
    st.N = spec.N
    st.node_set = spec.node_set
    st.n_par = spec.n_par
    st.n_perp = spec.n_perp
    st.face_id_static = _i(keep.fs)
    st.face_id_moving = _i(keep.fm)
    st.n_face_static = spec.n_face_static
    st.n_face_moving = spec.n_face_moving
    st.physics = spec.physics
    st.riemann = spec.riemann
    st.gamma = spec.gamma
    st.mu = spec.mu
    st.Pr = spec.Pr
    for d in range(3):
        st.normal[d] = float(spec.normal[d])
    st.dS = float(spec.dS)
    if getattr(spec, "metrics", None) is not None:
        keep.met = _f64(spec.metrics)
        st.metrics = _d(keep.met)
    else:
        st.metrics = None
    keep.st = st
    return keep


def mortar_flux(spec, n: int, s: float, Us, Um, Gs=None, Gm=None, rows=None, threads=1):
    """Whole operator (FP64).  Us/Um: [5][P][n_face], Gs/Gm: [3][5][P][n_face] or None.
    rows=(r0, r1) restricts the work to those rows (other columns of the outputs are 0).
    threads > 1 splits the rows into that many contiguous ranges and runs the same C
    routine on each range in its own thread (rows are independent periodic chains and
    write disjoint face columns; ctypes releases the GIL during the call)."""
    P = (spec.N + 1) ** 2
    Us, Um = _f64(Us), _f64(Um)
    Fs = np.zeros((5, P, spec.n_face_static))
    Fm = np.zeros((5, P, spec.n_face_moving))
    keep = _iface(spec)
    gs = _f64(Gs) if Gs is not None else None
    gm = _f64(Gm) if Gm is not None else None
    r0, r1 = (0, spec.n_perp) if rows is None else rows

    def run(a, b):
        return lib().orc_mortar_flux(C.byref(keep.st), n, s, _d(Us), _d(Um),
                                     _d(gs) if gs is not None else None,
                                     _d(gm) if gm is not None else None,
                                     _d(Fs), _d(Fm), a, b)

    threads = max(1, min(int(threads), r1 - r0))
    if threads == 1:
        rcs = [run(r0, r1)]
    else:
        from concurrent.futures import ThreadPoolExecutor
        cuts = [r0 + (r1 - r0) * k // threads for k in range(threads + 1)]
        with ThreadPoolExecutor(threads) as ex:
            rcs = list(ex.map(run, cuts[:-1], cuts[1:]))
    for rc in rcs:
        if rc:
            raise RuntimeError(f"oracle mortar_flux failed ({rc})")
    return Fs, Fm


def mortar_lifting(spec, n: int, s: float, Us, Um, rows=None, threads=1):
    """BR1 lifting surface term through the same operator (FP64): for each normal
    component d the mean of both mortar states times n_d dS, projected back onto both
    sides.  Returns Ls, Lm of shape [3][5][P][n_face]."""
    import copy
    comp = []
    for d in range(3):
        sp = copy.copy(spec)
        sp.physics, sp.riemann = EULER, LIFT + d
        comp.append(mortar_flux(sp, n, s, Us, Um, rows=rows, threads=threads))
    return np.stack([c[0] for c in comp]), np.stack([c[1] for c in comp])


def sort_mortars(tuples, m_col0: int, m_cols: int):
    t = np.ascontiguousarray(tuples, dtype=np.int32)
    count = t.shape[0]
    A = np.zeros((5, count), dtype=np.int32)
    m = np.zeros((2, m_cols), dtype=np.int32)
    rc = lib().orc_sort_mortars(count, _i(t), _i(A), _i(m), m_col0, m_cols)
    if rc:
        raise ValueError(f"sort failed ({rc})")
    return A, m


def index_map(side: int, n_par: int, n_perp: int, n: int, face_id, n_face: int, owner_opp=None):
    f = np.ascontiguousarray(face_id, dtype=np.int32).ravel()
    o = None if owner_opp is None else np.ascontiguousarray(owner_opp, dtype=np.int32).ravel()
    count = 2 * n_par * n_perp
    A = np.zeros((5, count), dtype=np.int32)
    m = np.zeros((2, n_face), dtype=np.int32)
    rc = lib().orc_index_map(side, n_par, n_perp, n, _i(f), n_face,
                             _i(o) if o is not None else None, _i(A), _i(m))
    if rc:
        raise ValueError(f"index map failed ({rc})")
    return A, m


def conservation(spec, Fs, Fm):
    """Returns an array [5][3]: static sum, moving sum, sum of |terms| per variable."""
    keep = _iface(spec)
    Fs, Fm = _f64(Fs), _f64(Fm)
    out = np.zeros((5, 3))
    lib().orc_conservation(C.byref(keep.st), _d(Fs), _d(Fm), _d(out))
    return out

"""CPU-side checks of the HIP library: it loads, exports every symbol that
include/mortar.h declares, and its host-only logic (validation, error strings, the FP64
displacement split) behaves; none of these calls touch a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2008_04356_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mortar.h")
LIB = os.path.join(ROOT, "paper_2008_04356_amd", "libmortar.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mortar_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (paper_2008_04356_amd/build.py)"
    lib = C.CDLL(LIB)
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


@pytest.fixture(scope="module")
def M():
    from paper_2008_04356_amd import mortar
    return mortar


def test_error_strings(M):
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(M.mortar_error_string(code), str)
    assert M.mortar_error_string(0) == "ok"


def test_decompose_matches_oracle_bitwise(M):
    rng = np.random.default_rng(0)
    cases = [0.0, -0.0, -1e-20, 3.0, 2.999, -0.4, 123.456, 1e-300, -1e-300]
    cases += list(rng.uniform(-1e5, 1e5, 2000)) + list(rng.uniform(-2, 2, 2000))
    for l in (1.0, 1.0 / 128, 2 * np.pi / 512, 0.37):
        for d in cases:
            dd = d * l if abs(d) < 1e6 else d
            assert M.mortar_decompose_displacement(dd, l) == O.decompose(dd, l)
    for bad in (np.nan, np.inf, -np.inf):
        with pytest.raises(M.MortarError):
            M.mortar_decompose_displacement(bad, 1.0)
    with pytest.raises(M.MortarError):
        M.mortar_decompose_displacement(1.0, 0.0)


def _desc(M, **kw):
    spec = W.make_plane(3, 8, 4, physics=W.NS, riemann=W.ROE, mu=1e-4)
    for k, v in kw.items():
        setattr(spec, k, v)
    return M.make_desc(spec)


def test_validation_errors_without_gpu(M):
    assert M.mortar_validate([_desc(M)]) == M.OK
    assert M.mortar_validate([_desc(M, N=0)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, N=12)]) == M.OK
    assert M.mortar_validate([_desc(M, N=15)]) == M.OK
    assert M.mortar_validate([_desc(M, N=16)]) == M.ERR_UNSUPPORTED
    # degrees above 9: no bf16/fp16 projection modes
    assert M.mortar_validate([_desc(M, N=10, precision=M.BF16_MFMA)]) == M.ERR_UNSUPPORTED
    assert M.mortar_validate([_desc(M, N=9, precision=M.BF16_MFMA)]) == M.OK
    assert M.mortar_validate([_desc(M, n_par=0)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, physics=7)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, riemann=3)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, node_set=2)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, precision=9)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, l_par=-1.0)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, l_par=float("nan"))]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, gamma=1.0)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, mu=-1.0)]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, normal=(1.0, 1.0, 0.0))]) == M.ERR_INVALID_ARG
    assert M.mortar_validate([_desc(M, n_face_static=10)]) == M.ERR_INVALID_ARG
    dup = np.arange(32, dtype=np.int32).reshape(4, 8)
    dup[1, 1] = dup[0, 0]
    assert M.mortar_validate([_desc(M, face_id_static=dup)]) == M.ERR_INVALID_ARG
    oob = np.arange(32, dtype=np.int32).reshape(4, 8)
    oob[3, 7] = 32
    assert M.mortar_validate([_desc(M, face_id_moving=oob)]) == M.ERR_INVALID_ARG
    many = np.arange(32 * 64, dtype=np.int32)[:32].reshape(4, 8) * 0 + np.arange(32).reshape(4, 8)
    assert M.mortar_validate([_desc(M, owner_static=many)]) == M.OK
    assert M.mortar_validate([]) == M.ERR_INVALID_ARG


@pytest.mark.parametrize("node_set", [0, 1])
def test_library_node_sets(M, node_set):
    """The library's own node routine (bracketing + bisection) against the oracle's
    (Newton) and numpy's, for every supported degree."""
    for N in range(1, 16):
        x, w = M.mortar_basis(N, node_set)
        xo, wo = O.nodes(N, node_set)
        assert np.max(np.abs(x - xo)) < 4e-16 and np.max(np.abs(w - wo)) < 4e-15
        if node_set == 0:
            xn, wn = np.polynomial.legendre.leggauss(N + 1)
            assert np.max(np.abs(x - xn)) < 4e-16
    with pytest.raises(M.MortarError):
        M.mortar_basis(16, node_set)
    with pytest.raises(M.MortarError):
        M.mortar_basis(0, node_set)


def test_binding_rejects_bad_face_arrays_before_the_library(M):
    """The convenience layer checks every tensor against the interface before the C ABI
    sees a pointer (the kernels address exactly [5][P][n_face] / [3][5][P][n_face] of
    the interface's element type): CPU tensors, wrong dtype, wrong shape, views that are
    not contiguous, missing gradients and wrong displacement counts are refused."""
    import torch
    ns = W.make_plane(2, 4, 2, physics=W.NS, riemann=W.ROE, mu=1e-3, precision=W.FP32)
    eu = W.make_plane(2, 4, 2, physics=W.EULER, riemann=W.LF, precision=W.FP64)
    P = ns.P
    st = torch.zeros((5, P, ns.n_face_static), dtype=torch.float32)
    gr = torch.zeros((3, 5, P, ns.n_face_static), dtype=torch.float32)
    with pytest.raises(M.MortarError, match="CUDA"):
        M._check_flux_args([ns], [st], [st], [gr], [gr], [st], [st])
    with pytest.raises(M.MortarError, match="missing"):
        M._check_list(None, [ns], "grad", "G_s")
    with pytest.raises(M.MortarError, match="entries"):
        M._check_list([st], [ns, ns], "state", "U_s")
    # Euler interfaces take no gradients
    M._check_list(None, [eu], "grad", "G_s")
    M._check_list([None], [eu], "grad", "G_s")

    class FakeCuda:
        """Stands in for a device tensor (no GPU here): only the checked attributes."""
        def __init__(self, shape, dtype, contiguous=True):
            self.shape, self.dtype, self.is_cuda, self._c = shape, dtype, True, contiguous

        def is_contiguous(self):
            return self._c

    ok = FakeCuda((5, P, ns.n_face_static), torch.float32)
    M._check_tensor(ok, ns, (5, P, ns.n_face_static), "F_s[0]")
    with pytest.raises(M.MortarError, match="dtype"):
        M._check_tensor(FakeCuda((5, P, ns.n_face_static), torch.float64), ns, ok.shape, "F_s[0]")
    with pytest.raises(M.MortarError, match="shape"):
        M._check_tensor(FakeCuda((5, P, ns.n_face_static - 1), torch.float32), ns, ok.shape, "F_s[0]")
    with pytest.raises(M.MortarError, match="contiguous"):
        M._check_tensor(FakeCuda(ok.shape, torch.float32, contiguous=False), ns, ok.shape, "F_s[0]")
    with pytest.raises(M.MortarError, match="displacements"):
        M._check_disp([0.1, 0.2], [ns], "mortar_update_displacement")

"""Driver of the DGSEM embedding (libdgembed.so, C ABI in include/dg_embed.h): a periodic
Cartesian box whose central slab slides along x1, the compressible Euler equations, and
the two sliding planes' fluxes from the mortar operator (libmortar.so), every Runge-Kutta
stage.  Argument marshalling and the time loop only: every operation on the solution runs
in the two HIP libraries.

The convergence test of the paper's Sec. 5.2 (errors of order N + 1 on a planar sliding
interface) is reproduced with a travelling density wave instead of the paper's manufactured
solution (which the paper cites but does not print): rho = rho0 + amp sin(2 pi (x1 + x2 +
x3 - 3 u0 t) / L) carried by the uniform velocity (u0, u0, u0) at constant pressure solves
the Euler equations without a source term; for Navier-Stokes (mu > 0) its heat flux is
balanced by an energy source the solver adds.  Navier-Stokes stages also run the
operator's lifting term (mortar_lifting) for the first Bassi-Rebay gradients and pass the
lifted face gradients to its flux.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import mortar as M
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgembed.so")

_dp = C.POINTER(C.c_double)


class dg_grid(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("j_lo", C.c_int32), ("j_hi", C.c_int32),
                ("L", C.c_double), ("vg", C.c_double), ("gamma", C.c_double),
                ("rho0", C.c_double), ("amp", C.c_double), ("u0", C.c_double), ("p0", C.c_double),
                ("basis", C.c_void_p), ("mu", C.c_double), ("Pr", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2008_04356_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.dg_basis_bytes.argtypes = [C.c_int]
    L.dg_basis_bytes.restype = C.c_int64
    L.dg_basis_tables.argtypes = [C.c_int, _dp]
    L.dg_exact_state.argtypes = [C.POINTER(dg_grid), C.c_double, vp, vp]
    L.dg_face_fluxes.argtypes = [C.POINTER(dg_grid), vp, vp, vp, vp]
    L.dg_face_states.argtypes = [C.POINTER(dg_grid), vp, vp, vp]
    L.dg_gradients.argtypes = [C.POINTER(dg_grid), vp, vp, vp, vp, vp, vp, vp, vp]
    L.dg_prolong_interface_gradients.argtypes = [C.POINTER(dg_grid), vp, vp, vp, vp, vp, vp]
    L.dg_prolong_interfaces.argtypes = [C.POINTER(dg_grid), vp, vp, vp, vp, vp, vp]
    L.dg_rhs.argtypes = [C.POINTER(dg_grid), vp, vp, vp, vp, vp, vp, vp, C.c_double, vp, vp]
    L.dg_rk_stage.argtypes = [vp, vp, vp, C.c_double, C.c_double, C.c_double, C.c_int64, vp]
    L.dg_density_error.argtypes = [C.POINTER(dg_grid), vp, C.c_double, vp, vp]
    return L


lib = _load()

# Low-storage Runge-Kutta of Carpenter and Kennedy (1994), five stages, fourth order:
# R = a_s R + dt RHS(U, t + c_s dt); U = U + b_s R.
RK_A = [0.0, -567301805773 / 1357537059087, -2404267990393 / 2016746695238,
        -3550918686646 / 2091501179385, -1275806237668 / 842570457699]
RK_B = [1432997174477 / 9575080441755, 5161836677717 / 13612068292357,
        1720146321549 / 2090206949498, 3134564353537 / 4481467310338,
        2277821191437 / 14882151754819]
RK_C = [0.0, 1432997174477 / 9575080441755, 2526269341429 / 6820363962896,
        2006345519317 / 3224310063776, 2802321613138 / 2924317926251]


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed ({rc})")


class SlidingBox:
    """The periodic box [0, L]^3 with K^3 elements of degree N; element layers
    K/3 <= j < 2K/3 along x2 slide along x1 with velocity vg."""

    def __init__(self, N, K, L=2.0, vg=1.0, gamma=1.4, rho0=1.0, amp=0.1, u0=0.5, p0=1.0 / 1.4,
                 mu=0.0, Pr=0.72, riemann=W.LF, node_set=W.GAUSS):
        import torch
        if K % 3:
            raise ValueError("K must be a multiple of 3 (slab between x2 = L/3 and 2L/3)")
        self.N, self.K, self.L, self.vg = N, K, L, vg
        self.h = L / K
        NP = N + 1
        self.NP = NP
        tab = np.zeros(lib.dg_basis_bytes(N) // 8)
        _check(lib.dg_basis_tables(N, tab.ctypes.data_as(_dp)), "dg_basis_tables")
        self.tab = torch.from_numpy(tab).cuda()
        self.g = dg_grid(N, K, K // 3, 2 * K // 3, L, vg, gamma, rho0, amp, u0, p0,
                         C.c_void_p(self.tab.data_ptr()), mu, Pr)
        self.ns = mu > 0.0
        n_elem = K ** 3
        dev = dict(dtype=torch.float64, device="cuda")
        self.U = torch.zeros((n_elem, 5, NP ** 3), **dev)
        self.R = torch.zeros_like(self.U)
        self.dU = torch.zeros_like(self.U)
        self.FF = torch.zeros((3, n_elem, 5, NP * NP), **dev)
        self.face = [[torch.zeros((5, NP * NP, K * K), **dev) for _ in range(2)] for _ in range(2)]
        self.flux = [[torch.zeros((5, NP * NP, K * K), **dev) for _ in range(2)] for _ in range(2)]
        self.err = torch.zeros(n_elem, **dev)
        if self.ns:
            self.UF = torch.zeros_like(self.FF)
            self.Q = torch.zeros((n_elem, 3, 5, NP ** 3), **dev)
            self.lift = [[torch.zeros((3, 5, NP * NP, K * K), **dev) for _ in range(2)] for _ in range(2)]
            self.grad = [[torch.zeros((3, 5, NP * NP, K * K), **dev) for _ in range(2)] for _ in range(2)]
        # both sliding planes: the layer below is the operator's static side (normal +e2),
        # the layer above its moving side; the flux is the plain normal flux (dS = 1)
        ids = np.arange(K * K, dtype=np.int32).reshape(K, K)   # column i + K k
        specs = []
        for name in ("lower plane", "upper plane"):
            spec = W.InterfaceSpec(N=N, n_par=K, n_perp=K, l_par=self.h, node_set=node_set,
                                   geometry=W.PLANE, physics=W.NS if mu > 0.0 else W.EULER,
                                   riemann=riemann, precision=W.FP64, gamma=gamma, mu=mu, Pr=Pr,
                                   normal=(0.0, 1.0, 0.0), dS=1.0,
                                   face_id_static=ids, face_id_moving=ids.copy(),
                                   n_face_static=K * K, n_face_moving=K * K, name=name)
            specs.append(spec)
        self.op = M.MortarOperator(specs)
        self.t = 0.0
        self.st = torch.cuda.current_stream().cuda_stream

    def close(self):
        self.op.close()

    def displacements(self, t):
        # lower plane: the slab (above) moves +vg t; upper plane: the static domain (above)
        # moves -vg t relative to the slab (below)
        return [self.vg * t, -self.vg * t]

    def set_exact(self, t=0.0):
        _check(lib.dg_exact_state(C.byref(self.g), t, C.c_void_p(self.U.data_ptr()), C.c_void_p(self.st)),
               "dg_exact_state")
        self.R.zero_()
        self.t = t

    def rhs(self, t):
        g, st = C.byref(self.g), C.c_void_p(self.st)
        p = lambda x: C.c_void_p(x.data_ptr())  # noqa: E731
        _check(lib.dg_prolong_interfaces(g, p(self.U), p(self.face[0][0]), p(self.face[0][1]),
                                         p(self.face[1][0]), p(self.face[1][1]), st), "dg_prolong_interfaces")
        self.op.update(self.displacements(t))
        Us, Um = [self.face[0][0], self.face[1][0]], [self.face[0][1], self.face[1][1]]
        Gs = Gm = None
        Q = None
        if self.ns:
            # first Bassi-Rebay: the sliding planes' lifting terms from the operator, the
            # conforming faces' averages here, then the gradients and their face values
            self.op.lifting(Us, Um, [self.lift[0][0], self.lift[1][0]], [self.lift[0][1], self.lift[1][1]])
            _check(lib.dg_face_states(g, p(self.U), p(self.UF), st), "dg_face_states")
            _check(lib.dg_gradients(g, p(self.U), p(self.UF), p(self.lift[0][0]), p(self.lift[0][1]),
                                    p(self.lift[1][0]), p(self.lift[1][1]), p(self.Q), st), "dg_gradients")
            _check(lib.dg_prolong_interface_gradients(g, p(self.Q), p(self.grad[0][0]), p(self.grad[0][1]),
                                                      p(self.grad[1][0]), p(self.grad[1][1]), st),
                   "dg_prolong_interface_gradients")
            Gs, Gm = [self.grad[0][0], self.grad[1][0]], [self.grad[0][1], self.grad[1][1]]
            Q = p(self.Q)
        self.op.flux(Us, Um, Gs, Gm, [self.flux[0][0], self.flux[1][0]], [self.flux[0][1], self.flux[1][1]])
        _check(lib.dg_face_fluxes(g, p(self.U), Q, p(self.FF), st), "dg_face_fluxes")
        _check(lib.dg_rhs(g, p(self.U), Q, p(self.FF), p(self.flux[0][0]), p(self.flux[0][1]),
                          p(self.flux[1][0]), p(self.flux[1][1]), t, p(self.dU), st), "dg_rhs")

    def step(self, dt):
        n = self.U.numel()
        for s in range(5):
            self.rhs(self.t + RK_C[s] * dt)
            _check(lib.dg_rk_stage(C.c_void_p(self.U.data_ptr()), C.c_void_p(self.R.data_ptr()),
                                   C.c_void_p(self.dU.data_ptr()), RK_A[s], RK_B[s], dt, n,
                                   C.c_void_p(self.st)), "dg_rk_stage")
        self.t += dt

    def stable_dt(self, cfl=0.5):
        g = self.g
        c = math.sqrt(g.gamma * g.p0 / (g.rho0 - g.amp))
        lam = math.sqrt(3.0) * abs(g.u0) + abs(self.vg) + c
        dt = cfl * self.h / ((2 * self.N + 1) * lam)
        if self.ns:
            # the viscous limit: diffusivity max(mu, k / c_v) / rho over (h / (N + 1)^2)^2
            nu = max(g.mu, g.mu * g.gamma / g.Pr) / (g.rho0 - g.amp)
            dt = min(dt, cfl * (self.h / (self.N + 1) ** 2) ** 2 / nu)
        return dt

    def run(self, t_end, cfl=0.5):
        steps = max(1, int(math.ceil(t_end / self.stable_dt(cfl) - 1e-12)))
        dt = t_end / steps
        for _ in range(steps):
            self.step(dt)
        return steps

    def density_l2_error(self):
        import torch
        _check(lib.dg_density_error(C.byref(self.g), C.c_void_p(self.U.data_ptr()), self.t,
                                    C.c_void_p(self.err.data_ptr()), C.c_void_p(self.st)), "dg_density_error")
        torch.cuda.synchronize()
        return float(math.sqrt(float(np.sum(self.err.cpu().numpy()))))


def convergence(N, Ks, t_end=1.0, cfl=0.5, **kw):
    """L2 density errors at t_end and the observed orders log2(e_coarse / e_fine)."""
    errs = []
    for K in Ks:
        box = SlidingBox(N, K, **kw)
        try:
            box.set_exact(0.0)
            box.run(t_end, cfl)
            errs.append(box.density_l2_error())
        finally:
            box.close()
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(Ks[i + 1] / Ks[i]) for i in range(len(errs) - 1)]
    return errs, orders

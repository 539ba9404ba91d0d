"""Seeded synthetic workloads for the sliding-mesh mortar operator.

This module describes interfaces and generates face data; it contains none of the
operator's arithmetic (no projections, no fluxes, no pairing).  Both the GPU path's
tests/benchmark and the CPU oracle consume what it produces.

Face data are samples of smooth analytic fields at the face nodes (node positions come
from numpy's Legendre routines), plus a small independent per-point "DG jump" noise,
so that the two sides of the interface disagree slightly as discontinuous Galerkin
traces do.  The paper's own workloads (a rotating vortex, a manufactured solution and
a turbine LES, Sec. 5) need a full solver and external meshes; these fields stand in
for them with the same shapes: free stream rho = 1, normal velocity 0.3, p = 0.71
(Mach about 0.3), gamma = 1.4, small smooth perturbations.

Interface shapes (Fig. of the possible 3D interface geometries): plane, plane annular
axial, and surfaces of revolution (cylindrical radial, conical) with polynomial face
geometry.

Layouts: U[5][P][n_face], G[3][5][P][n_face] (G[d][v] = dU_v/dx_d), metrics
M[4][P][n_face] = (nx, ny, nz, dS); point p = p_par + (N+1) * p_perp; the face of
(i_par, i_perp) sits in column face_id[i_perp, i_par].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

GAUSS, LGL = 0, 1
EULER, NS = 0, 1
LF, ROE = 0, 1
PLANE, ANNULUS, REVOLUTION = 0, 1, 2
FP64, FP32, BF16_MFMA, FP16_MFMA = 0, 1, 2, 3

FREE_STREAM = dict(rho=1.0, vn=0.3, p=0.71)


@dataclasses.dataclass
class InterfaceSpec:
    N: int
    n_par: int
    n_perp: int
    l_par: float
    node_set: int = GAUSS
    geometry: int = PLANE
    physics: int = EULER
    riemann: int = LF
    precision: int = FP64
    gamma: float = 1.4
    mu: float = 0.0
    Pr: float = 0.72
    normal: tuple = (1.0, 0.0, 0.0)
    dS: float = 1.0
    metrics: Optional[np.ndarray] = None           # [4][P][n_face_static] or None
    face_id_static: Optional[np.ndarray] = None    # [n_perp, n_par] int32
    face_id_moving: Optional[np.ndarray] = None
    n_face_static: int = 0
    n_face_moving: int = 0
    owner_static: Optional[np.ndarray] = None      # [n_perp, n_par] int32 or None
    owner_moving: Optional[np.ndarray] = None
    r_edges: Optional[np.ndarray] = None           # annulus radii / generatrix edges [n_perp + 1]
    beta: float = 0.0                              # surface of revolution: cone half-angle
    r0: float = 1.0                                # surface of revolution: radius at s = 0
    name: str = ""

    @property
    def NP(self) -> int:
        return self.N + 1

    @property
    def P(self) -> int:
        return (self.N + 1) ** 2

    @property
    def n_pairs(self) -> int:
        return self.n_par * self.n_perp

    @property
    def mortar_points(self) -> int:
        return 2 * self.n_pairs * self.P

    @property
    def n_in_vars(self) -> int:
        return 20 if self.physics == NS else 5


def node_positions(N: int, node_set: int) -> np.ndarray:
    """Reference node positions from numpy's Legendre routines."""
    if node_set == GAUSS:
        x, _ = np.polynomial.legendre.leggauss(N + 1)
        return x
    inner = np.polynomial.legendre.Legendre.basis(N).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def synthetic_face_ids(n_par: int, n_perp: int, scramble_seed: Optional[int] = None,
                       extra_cols: int = 0):
    """Columns for every face: i_par + n_par * i_perp (coalesced), or a seeded permutation
    over n_par*n_perp + extra_cols columns (exercises the indirection and unused columns)."""
    nf = n_par * n_perp
    if scramble_seed is None and extra_cols == 0:
        ids = np.arange(nf, dtype=np.int32).reshape(n_perp, n_par)
        return ids, nf
    rng = np.random.Generator(np.random.PCG64(scramble_seed if scramble_seed is not None else 0))
    cols = rng.permutation(nf + extra_cols)[:nf].astype(np.int32)
    return cols.reshape(n_perp, n_par), nf + extra_cols


def make_plane(N: int, n_par: int, n_perp: int, physics: int = EULER, riemann: int = LF,
               precision: int = FP64, node_set: int = GAUSS, mu: float = 0.0,
               scramble_seed: Optional[int] = None, extra_cols: int = 0,
               name: str = "") -> InterfaceSpec:
    """Plane interface: normal e_x, sliding along e_y (parallel), e_z across; the interface
    is periodic with unit period in y and z."""
    l_par, l_perp = 1.0 / n_par, 1.0 / n_perp
    fs, nfs = synthetic_face_ids(n_par, n_perp, scramble_seed, extra_cols)
    fm, nfm = synthetic_face_ids(n_par, n_perp,
                                 None if scramble_seed is None else scramble_seed + 7, extra_cols)
    return InterfaceSpec(N=N, n_par=n_par, n_perp=n_perp, l_par=l_par, node_set=node_set,
                         geometry=PLANE, physics=physics, riemann=riemann, precision=precision,
                         mu=mu, normal=(1.0, 0.0, 0.0), dS=l_par * l_perp / 4.0,
                         face_id_static=fs, face_id_moving=fm, n_face_static=nfs,
                         n_face_moving=nfm, name=name)


def make_annulus(N: int, n_par: int, n_perp: int, seed: int, physics: int = NS,
                 riemann: int = ROE, precision: int = FP32, node_set: int = GAUSS,
                 mu: float = 1e-4, r_in: float = 0.8, r_out: float = 1.0,
                 name: str = "") -> InterfaceSpec:
    """Plane annular axial interface: normal e_z, sliding in theta (l_par in radians),
    radial rows with seeded jittered edges in [r_in, r_out].  Static metrics per point:
    n = e_z and dS = r * (l_par/2) * (dr_j/2)."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    l_par = 2.0 * math.pi / n_par
    j = np.arange(n_perp + 1, dtype=np.float64)
    jitter = rng.uniform(-0.3, 0.3, n_perp + 1)
    jitter[0] = jitter[-1] = 0.0
    r_edges = r_in + (r_out - r_in) * (j + jitter) / n_perp
    fs, nfs = synthetic_face_ids(n_par, n_perp)
    fm, nfm = synthetic_face_ids(n_par, n_perp)
    x = node_positions(N, node_set)
    NP = N + 1
    P = NP * NP
    met = np.zeros((4, P, nfs))
    for ip in range(n_perp):
        dr = r_edges[ip + 1] - r_edges[ip]
        for pp in range(NP):
            r = r_edges[ip] + 0.5 * (x[pp] + 1.0) * dr
            for pa in range(NP):
                p = pa + NP * pp
                cols = fs[ip, :]
                met[2, p, cols] = 1.0
                met[3, p, cols] = r * (l_par / 2.0) * (dr / 2.0)
    return InterfaceSpec(N=N, n_par=n_par, n_perp=n_perp, l_par=l_par, node_set=node_set,
                         geometry=ANNULUS, physics=physics, riemann=riemann,
                         precision=precision, mu=mu, normal=(0.0, 0.0, 1.0), dS=0.0,
                         metrics=met, face_id_static=fs, face_id_moving=fm,
                         n_face_static=nfs, n_face_moving=nfm, r_edges=r_edges, name=name)


def revolution_point(beta: float, r0: float, th, s):
    """Point of the surface of revolution at angle th and generatrix coordinate s:
    (r cos th, r sin th, z) with r = r0 + s sin(beta), z = s cos(beta).  beta = 0 is the
    cylinder r = r0 (cylindrical radial interface), 0 < beta < pi/2 a cone (conical
    interface), beta = pi/2 the flat annulus z = 0."""
    r = r0 + s * math.sin(beta)
    return np.stack(np.broadcast_arrays(r * np.cos(th), r * np.sin(th), s * math.cos(beta)))


def revolution_frame(beta: float, th):
    """Unit tangents along the slide (e_th) and the generatrix (e_s), and the normal
    n = e_s x e_th (the cylinder's points to the axis, the flat annulus's is +e_z)."""
    ct, st = np.cos(th), np.sin(th)
    sb, cb = math.sin(beta), math.cos(beta)
    e_th = np.stack([-st, ct, np.zeros_like(th)])
    e_s = np.stack([sb * ct, sb * st, np.full_like(th, cb)])
    n = np.stack([e_s[1] * e_th[2] - e_s[2] * e_th[1],
                  e_s[2] * e_th[0] - e_s[0] * e_th[2],
                  e_s[0] * e_th[1] - e_s[1] * e_th[0]])
    return e_th, e_s, n


def make_revolution(N: int, n_par: int, n_perp: int, beta: float, seed: int,
                    physics: int = NS, riemann: int = ROE, precision: int = FP32,
                    node_set: int = GAUSS, mu: float = 1e-4, r0: float = 1.0,
                    length: float = 0.5, exact_metrics: bool = False,
                    name: str = "") -> InterfaceSpec:
    """Curved interface on a surface of revolution (cylindrical radial for beta = 0,
    conical for 0 < beta < pi/2), sliding in theta (l_par in radians), rows along the
    generatrix with seeded jittered edges in [0, length].

    Each static face is the degree-N polynomial through the exact surface points at its
    nodes (the face geometry of a high-order mesh).  Its nodal metrics come from that
    polynomial: a = dX/d(eta) x dX/d(xi) at the node, n = a / |a|, dS = |a|.  With
    exact_metrics the nodal metrics are the exact surface's instead: n = e_s x e_th,
    dS = r (l_par/2) (ds/2)."""
    rng = np.random.Generator(np.random.PCG64(2000 + seed))
    l_par = 2.0 * math.pi / n_par
    j = np.arange(n_perp + 1, dtype=np.float64)
    jitter = rng.uniform(-0.3, 0.3, n_perp + 1)
    jitter[0] = jitter[-1] = 0.0
    s_edges = length * (j + jitter) / n_perp
    fs, nfs = synthetic_face_ids(n_par, n_perp)
    fm, nfm = synthetic_face_ids(n_par, n_perp)
    x = node_positions(N, node_set)
    NP, P = N + 1, (N + 1) ** 2
    # derivatives of the nodal interpolant at the nodes: D[a, b] = l_b'(x_a), from
    # numpy's Legendre fit of the cardinal functions
    leg = np.polynomial.legendre
    D = leg.legval(x, leg.legder(leg.legfit(x, np.eye(NP), N))).T
    met = np.zeros((4, P, nfs))
    for ip in range(n_perp):
        ds = s_edges[ip + 1] - s_edges[ip]
        sv = s_edges[ip] + 0.5 * (x + 1.0) * ds                       # [NP] along eta
        for i in range(n_par):
            th = (i + 0.5 * (x + 1.0)) * l_par                         # [NP] along xi
            TH, SV = np.meshgrid(th, sv)                               # [pp, pa]
            if exact_metrics:
                _, _, n = revolution_frame(beta, TH)
                dS = (r0 + SV * math.sin(beta)) * (l_par / 2.0) * (ds / 2.0)
            else:
                X = revolution_point(beta, r0, TH, SV)                 # [3, pp, pa]
                Xxi = np.einsum("ab,cpb->cpa", D, X)
                Xeta = np.einsum("ab,cbq->caq", D, X)
                a = np.cross(Xeta, Xxi, axis=0)
                dS = np.sqrt(np.sum(a * a, axis=0))
                n = a / dS
            cols = fs[ip, i]
            for pp in range(NP):
                for pa in range(NP):
                    p = pa + NP * pp
                    met[0:3, p, cols] = n[:, pp, pa]
                    met[3, p, cols] = dS[pp, pa]
    return InterfaceSpec(N=N, n_par=n_par, n_perp=n_perp, l_par=l_par, node_set=node_set,
                         geometry=REVOLUTION, physics=physics, riemann=riemann,
                         precision=precision, mu=mu, normal=(0.0, 0.0, 1.0), dS=0.0,
                         metrics=met, face_id_static=fs, face_id_moving=fm,
                         n_face_static=nfs, n_face_moving=nfm, r_edges=s_edges, beta=beta,
                         r0=r0, name=name)


def seeded_owners(spec: InterfaceSpec, seed: int, n_static_ranks: int, n_moving_ranks: int):
    """Virtual ranks: contiguous blocks of faces along (i_perp, i_par) per rank, as a
    space-filling-curve partition would give on a structured interface."""
    rng = np.random.Generator(np.random.PCG64(5000 + seed))

    def part(nr):
        nf = spec.n_par * spec.n_perp
        cuts = np.sort(rng.choice(np.arange(1, nf), size=nr - 1, replace=False))
        own = np.zeros(nf, dtype=np.int32)
        for c in cuts:
            own[c:] += 1
        ranks = np.sort(rng.choice(np.arange(3 * nr), size=nr, replace=False)).astype(np.int32)
        return ranks[own].reshape(spec.n_perp, spec.n_par)

    spec.owner_static = part(n_static_ranks)
    spec.owner_moving = part(n_moving_ranks)
    return spec


# --------------------------------------------------------------------------------------
# Fields
# --------------------------------------------------------------------------------------

def _plane_field(rng, n_modes=3):
    """Per primitive variable: sum of sines with integer multiples of 2*pi in y and z."""
    k = np.zeros((n_modes, 3))
    k[:, 0] = rng.uniform(-3.0, 3.0, n_modes)
    k[:, 1] = 2.0 * math.pi * rng.integers(1, 4, n_modes)
    k[:, 2] = 2.0 * math.pi * rng.integers(1, 4, n_modes)
    amp = rng.uniform(0.5, 1.0, (5, n_modes)) * 1e-2
    phase = rng.uniform(0.0, 2.0 * math.pi, (5, n_modes))
    return k, amp, phase


def _eval_plane_prim(field, y, z, grad=True):
    """Primitive (rho, vx, vy, vz, p) and their gradients (None without grad) at x = 0,
    for y of shape [1, n_par, 1, NP] (the slide) and z of shape [n_perp, 1, NP, 1] (rows).
    Every mode is separable by the angle-sum rule, so the sums over modes are products
    of [rows x modes] and [modes x slide] tables."""
    k, amp, phase = field
    n_perp, _, NP, _ = z.shape
    n_par = y.shape[1]
    y1, z1 = y.reshape(-1), z.reshape(-1)
    B = np.outer(z1, k[:, 2])                        # [n_z, modes]
    sB, cB = np.sin(B), np.cos(B)
    base = np.array([FREE_STREAM["rho"], FREE_STREAM["vn"], 0.0, 0.0, FREE_STREAM["p"]])

    def grid(x):                                     # [n_z, n_y] -> [n_perp, n_par, NP, NP]
        return x.reshape(n_perp, NP, n_par, NP).transpose(0, 2, 1, 3)

    q = np.empty((5, n_perp, n_par, NP, NP))
    dq = np.empty((3, 5, n_perp, n_par, NP, NP)) if grad else None
    for v in range(5):
        A = np.outer(y1, k[:, 1]) + phase[v][None, :]    # [n_y, modes]
        sA, cA = np.sin(A) * amp[v], np.cos(A) * amp[v]
        q[v] = grid(base[v] + cB @ sA.T + sB @ cA.T)     # sum_m amp sin(A + B)
        if grad:
            for d in range(3):                           # sum_m amp k_d cos(A + B)
                dq[d, v] = grid((cB * k[:, d]) @ cA.T - (sB * k[:, d]) @ sA.T)
    return q, dq


def _annulus_field(rng, n_modes=32):
    m_theta = rng.integers(1, 33, n_modes)
    kr = rng.uniform(-20.0, 20.0, n_modes)
    kz = rng.uniform(-5.0, 5.0, n_modes)
    kmag = np.sqrt(m_theta.astype(float) ** 2 + kr ** 2)
    shape = kmag ** (-5.0 / 6.0)
    amp = rng.uniform(0.5, 1.0, (5, n_modes)) * shape[None, :]
    amp *= 1e-2 / np.sqrt(0.5 * np.sum(amp ** 2, axis=1, keepdims=True))  # rms 1e-2
    phase = rng.uniform(0.0, 2.0 * math.pi, (5, n_modes))
    return m_theta, kr, kz, amp, phase


def _eval_annulus_prim(field, r, th):
    """Primitive variables and gradients of the annulus field at radius r (shape
    [n_perp, 1, NP, 1]: rows and their nodes) and angle th (shape [1, n_par, 1, NP]: the
    slide).  Every mode is separable by the angle-sum rule, so the sums over modes are
    products of [rows x modes] and [modes x slide] tables."""
    m_theta, kr, kz, amp, phase = field
    n_perp, _, NP, _ = r.shape
    n_par = th.shape[1]
    r1, t1 = r.reshape(-1), th.reshape(-1)
    B = np.outer(r1 - 0.8, kr)                       # [n_r, modes]
    sB, cB = np.sin(B), np.cos(B)
    ct, st, ir = np.cos(t1)[None, :], np.sin(t1)[None, :], (1.0 / r1)[:, None]
    base = np.array([FREE_STREAM["rho"], 0.0, 0.0, FREE_STREAM["vn"], FREE_STREAM["p"]])

    def grid(x):                                     # [n_r, n_t] -> [n_perp, n_par, NP, NP]
        return x.reshape(n_perp, NP, n_par, NP).transpose(0, 2, 1, 3)

    q = np.empty((5, n_perp, n_par, NP, NP))
    dq = np.empty((3, 5, n_perp, n_par, NP, NP))
    for v in range(5):
        A = np.outer(t1, m_theta) + phase[v][None, :]     # [n_t, modes]
        sA, cA = np.sin(A) * amp[v], np.cos(A) * amp[v]
        # sum_m amp sin(A + B) and sum_m w_m amp cos(A + B)
        q[v] = grid(base[v] + cB @ sA.T + sB @ cA.T)

        def csum(w):
            return (cB * w) @ cA.T - (sB * w) @ sA.T
        x_r, x_t = csum(kr), csum(m_theta.astype(np.float64))
        dq[0, v] = grid(ct * x_r - (st * ir) * x_t)
        dq[1, v] = grid(st * x_r + (ct * ir) * x_t)
        dq[2, v] = grid(csum(kz))
    return q, dq


def _prim_to_cons(q, dq, gamma):
    rho, u, v, w, p = q
    vel = np.stack([u, v, w])
    U = np.empty_like(q)
    U[0] = rho
    U[1:4] = rho * vel
    U[4] = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel ** 2, axis=0)
    if dq is None:
        return U, None
    G = np.empty_like(dq)
    for d in range(3):
        drho, dvel, dp = dq[d, 0], dq[d, 1:4], dq[d, 4]
        G[d, 0] = drho
        G[d, 1:4] = vel * drho + rho * dvel
        G[d, 4] = dp / (gamma - 1.0) + 0.5 * np.sum(vel ** 2, axis=0) * drho \
            + rho * np.sum(vel * dvel, axis=0)
    return U, G


def make_inputs(spec: InterfaceSpec, seed: int, delta: float = 0.0, noise: float = 1e-4):
    """Face data for both sides (FP64 numpy).  The moving side is sampled at its
    positions displaced by delta along the sliding direction."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N, NP, P = spec.N, spec.NP, spec.P
    x = node_positions(N, spec.node_set)
    ia = np.arange(spec.n_par)[None, :, None, None]
    ip = np.arange(spec.n_perp)[:, None, None, None]
    xa = x[None, None, None, :]   # along
    xp = x[None, None, :, None]   # across
    out = {}
    if spec.geometry == PLANE:
        field = _plane_field(rng)
        l_perp = 1.0 / spec.n_perp
        for side, shift in (("s", 0.0), ("m", delta)):
            y = (ia + 0.5 * (xa + 1.0)) * spec.l_par + shift
            z = (ip + 0.5 * (xp + 1.0)) * l_perp
            q, dq = _eval_plane_prim(field, y, z, grad=spec.physics == NS)
            out[side] = _prim_to_cons(q, dq, spec.gamma)
    elif spec.geometry == REVOLUTION:
        field = _annulus_field(rng)
        se = spec.r_edges
        for side, shift in (("s", 0.0), ("m", delta)):
            th = (ia + 0.5 * (xa + 1.0)) * spec.l_par + shift
            sv = se[:-1][:, None, None, None] + 0.5 * (xp + 1.0) * np.diff(se)[:, None, None, None]
            # the annulus field with its radius running over [0.8, 1] along the generatrix;
            # its velocity components (x, y, z) become components along (e_th, e_s, n), so
            # the free stream crosses the interface with normal velocity 0.3 as elsewhere
            q, dq = _eval_annulus_prim(field, 0.8 + 0.2 * sv / se[-1], th)
            e_th, e_s, nrm = revolution_frame(spec.beta, th)   # broadcast over rows
            q[1:4] = q[1] * e_th + q[2] * e_s + q[3] * nrm
            for d in range(3):
                dq[d, 1:4] = dq[d, 1] * e_th + dq[d, 2] * e_s + dq[d, 3] * nrm
            out[side] = _prim_to_cons(q, dq, spec.gamma)
    else:
        field = _annulus_field(rng)
        re = spec.r_edges
        for side, shift in (("s", 0.0), ("m", delta)):
            th = (ia + 0.5 * (xa + 1.0)) * spec.l_par + shift
            r = re[:-1][:, None, None, None] + 0.5 * (xp + 1.0) * np.diff(re)[:, None, None, None]
            q, dq = _eval_annulus_prim(field, r, th)
            out[side] = _prim_to_cons(q, dq, spec.gamma)

    res = {}
    for side, fid, nf in (("s", spec.face_id_static, spec.n_face_static),
                          ("m", spec.face_id_moving, spec.n_face_moving)):
        U, G = out[side]  # U [5, n_perp, n_par, NP(perp), NP(par)], G [3, 5, ...]
        U = U + noise * rng.uniform(-1.0, 1.0, U.shape)
        Ua = np.zeros((5, P, nf))
        cols = fid.reshape(-1)
        # point p = p_par + NP * p_perp
        Ua[:, :, cols] = U.transpose(0, 3, 4, 1, 2).reshape(5, P, -1)
        del U
        Ga = None
        if G is not None:
            G = G + noise * rng.uniform(-1.0, 1.0, G.shape)
            Ga = np.zeros((3, 5, P, nf))
            Ga[:, :, :, cols] = G.transpose(0, 1, 4, 5, 2, 3).reshape(3, 5, P, -1)
        res["U" + side] = Ua
        res["G" + side] = Ga if spec.physics == NS else None
    return res


def constant_inputs(spec: InterfaceSpec, prim=(1.0, 0.3, 0.0, 0.0, 0.71)):
    """A constant state on both sides with zero gradients (free-stream check)."""
    rho, u, v, w, p = prim
    U = np.array([rho, rho * u, rho * v, rho * w,
                  p / (spec.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])
    res = {}
    for side, nf in (("s", spec.n_face_static), ("m", spec.n_face_moving)):
        res["U" + side] = np.repeat(np.repeat(U[:, None, None], spec.P, 1), nf, 2)
        res["G" + side] = np.zeros((3, 5, spec.P, nf)) if spec.physics == NS else None
    return res


def round_to(arr, precision: int):
    """Inputs as the GPU sees them: FP64, or FP32 for the FP32 and MFMA modes."""
    if arr is None:
        return None
    if precision == FP64:
        return np.asarray(arr, dtype=np.float64)
    return np.asarray(arr, dtype=np.float32)


# --------------------------------------------------------------------------------------
# The workloads: plane, annulus, turbine-like batch, precision stress, curved shapes
# --------------------------------------------------------------------------------------

def config(idx: int, precision: int = None):
    """Returns (list of InterfaceSpec, per-stage displacement function(stage) -> list)."""
    if idx == 1:
        spec = make_plane(3, 8, 8, physics=EULER, riemann=LF,
                          precision=FP64 if precision is None else precision, name="plane N=3 8x8")
        rng = np.random.Generator(np.random.PCG64(1))
        ns = rng.integers(0, 8, 10)
        ss = rng.uniform(0.0, 1.0, 10)

        def disp(k):
            return [float((ns[k % 10] + ss[k % 10]) * spec.l_par)]
        return [spec], disp
    if idx == 2:
        spec = make_plane(5, 128, 64, physics=NS, riemann=ROE, mu=1e-4,
                          precision=FP32 if precision is None else precision, name="plane N=5 128x64")

        def disp(k):
            return [0.0137 * k * spec.l_par]
        return [spec], disp
    if idx == 3:
        spec = make_annulus(7, 512, 64, seed=3,
                            precision=FP32 if precision is None else precision, name="annulus N=7 512x64")

        def disp(k):
            return [0.0137 * k * spec.l_par]
        return [spec], disp
    if idx == 4:
        p = FP32 if precision is None else precision
        specs = [make_annulus(7, 320, 125, seed=41, precision=p, name="annulus N=7 320x125"),
                 make_annulus(5, 256, 72, seed=42, precision=p, name="annulus N=5 256x72"),
                 make_plane(3, 64, 32, physics=NS, riemann=ROE, mu=1e-4, precision=p,
                            name="plane N=3 64x32")]
        speeds = [0.0137, 0.0211, 0.0093]

        def disp(k):
            return [speeds[i] * k * specs[i].l_par for i in range(3)]
        return specs, disp
    if idx in (6, 7):
        # curved interfaces at the annulus workload's size: cylindrical radial (6) and
        # conical with a 30 degree half-angle (7), polynomial face geometry
        spec = make_revolution(7, 512, 64, 0.0 if idx == 6 else math.pi / 6, seed=idx,
                               precision=FP32 if precision is None else precision,
                               name="cylinder N=7 512x64" if idx == 6 else "cone N=7 512x64")

        def disp(k):
            return [0.0137 * k * spec.l_par]
        return [spec], disp
    if idx == 5:
        spec = make_plane(9, 256, 256, physics=EULER, riemann=ROE,
                          precision=FP32 if precision is None else precision, name="plane N=9 256x256")

        def disp(k):
            return [0.0137 * k * spec.l_par]
        return [spec], disp
    raise ValueError(idx)

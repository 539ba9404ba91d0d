"""Pins of the oracle's pointwise fluxes (Sec. 2 Navier-Stokes fluxes; Sec. 3.1 Roe
solver with Harten-Hyman entropy fix and BR1 viscous flux; Lax-Friedrichs flux).

Absolute numerical-flux values have no printed reference in the paper; they are fixed
here by invariants: consistency, conservation in direction, rotational invariance,
Roe's exact resolution of isolated waves (contact, shear, Rankine-Hugoniot shock),
full upwinding in supersonic flow, and analytic viscous fluxes of linear fields."""
import math

import numpy as np
import pytest

from oracle import oracle as O

GAMMA = 1.4


def cons(rho, v, p):
    v = np.asarray(v, dtype=float)
    return np.array([rho, *(rho * v), p / (GAMMA - 1.0) + 0.5 * rho * v @ v])


def rand_state(rng):
    return cons(rng.uniform(0.5, 2.0), rng.uniform(-0.5, 0.5, 3), rng.uniform(0.5, 2.0))


def rand_normal(rng):
    n = rng.normal(size=3)
    return n / np.linalg.norm(n)


def rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("riemann", [O.LF, O.ROE])
def test_consistency(riemann):
    rng = np.random.default_rng(1)
    for _ in range(50):
        U, n = rand_state(rng), rand_normal(rng)
        F = O.point_flux(U, U, normal=n, riemann=riemann)
        assert np.max(np.abs(F - O.euler_normal_flux(U, n))) < 1e-14


@pytest.mark.parametrize("riemann", [O.LF, O.ROE])
def test_direction_antisymmetry_and_rotation(riemann):
    rng = np.random.default_rng(2)
    for _ in range(50):
        UL, UR, n, R = rand_state(rng), rand_state(rng), rand_normal(rng), rot(rng)
        F = O.point_flux(UL, UR, normal=n, riemann=riemann)
        G = O.point_flux(UR, UL, normal=-n, riemann=riemann)
        assert np.max(np.abs(F + G)) < 1e-14
        RU = lambda U: np.array([U[0], *(R @ U[1:4]), U[4]])  # noqa: E731
        Fr = O.point_flux(RU(UL), RU(UR), normal=R @ n, riemann=riemann)
        assert np.max(np.abs(Fr - RU(F))) < 1e-13


def _frame(n, rng):
    t = np.cross(n, rand_normal(rng))
    return t / np.linalg.norm(t)


def test_roe_contact_and_shear_upwind():
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = rand_normal(rng)
        t = _frame(n, rng)
        vt = rng.uniform(-0.3, 0.3)
        for vn in (0.2, -0.2):
            v = vn * n + vt * t
            UL, UR = cons(1.0, v, 0.8), cons(1.7, v, 0.8)  # contact: density jump only
            F = O.point_flux(UL, UR, normal=n, riemann=O.ROE)
            up = UL if vn > 0 else UR
            assert np.max(np.abs(F - O.euler_normal_flux(up, n))) < 1e-14
            UL, UR = cons(1.2, v, 0.8), cons(1.2, v + 0.25 * t, 0.8)  # shear only
            F = O.point_flux(UL, UR, normal=n, riemann=O.ROE)
            up = UL if vn > 0 else UR
            assert np.max(np.abs(F - O.euler_normal_flux(up, n))) < 1e-14


@pytest.mark.parametrize("Ms", [1.1, 1.5, 3.0])
def test_roe_resolves_rankine_hugoniot_shock(Ms):
    rng = np.random.default_rng(int(Ms * 10))
    for _ in range(10):
        n = rand_normal(rng)
        t = _frame(n, rng)
        vt = rng.uniform(-0.3, 0.3)
        rhoR, uR, pR = 1.0, rng.uniform(-0.2, 0.2), 0.71
        cR = math.sqrt(GAMMA * pR / rhoR)
        S = uR + Ms * cR                       # right-running shock into state R
        pL = pR * (1.0 + 2.0 * GAMMA / (GAMMA + 1.0) * (Ms * Ms - 1.0))
        rhoL = rhoR * (GAMMA + 1.0) * Ms * Ms / ((GAMMA - 1.0) * Ms * Ms + 2.0)
        uL = S - (S - uR) * rhoR / rhoL
        UL = cons(rhoL, uL * n + vt * t, pL)
        UR = cons(rhoR, uR * n + vt * t, pR)
        FL, FR = O.euler_normal_flux(UL, n), O.euler_normal_flux(UR, n)
        assert np.max(np.abs((FL - FR) - S * (UL - UR))) < 1e-12   # the data is a shock
        F = O.point_flux(UL, UR, normal=n, riemann=O.ROE)
        assert np.max(np.abs(F - FL)) < 1e-12 * max(1.0, np.max(np.abs(FL)))


@pytest.mark.parametrize("Ms", [1.05, 1.3, 2.0])
def test_roe_stationary_and_slow_shocks_keep_the_fix_off(Ms):
    """A transonic (stationary or slow) compressive shock: lambda_L > lambda~ > lambda_R;
    the entropy fix must not act, so Roe still returns the upwind flux exactly."""
    rng = np.random.default_rng(int(Ms * 100))
    for frac in (0.0, 0.02, -0.02):
        n = rand_normal(rng)
        rhoR, pR = 1.0, 0.71
        cR = math.sqrt(GAMMA * pR / rhoR)
        uR = -Ms * cR + frac * cR                 # shock speed S = frac * cR
        S = uR + Ms * cR
        pL = pR * (1.0 + 2.0 * GAMMA / (GAMMA + 1.0) * (Ms * Ms - 1.0))
        rhoL = rhoR * (GAMMA + 1.0) * Ms * Ms / ((GAMMA - 1.0) * Ms * Ms + 2.0)
        uL = S - (S - uR) * rhoR / rhoL
        # moving towards -n: the upwind side of the interface is R, its wave the u - c one
        UL = cons(rhoR, -uR * n, pR)
        UR = cons(rhoL, -uL * n, pL)
        F = O.point_flux(UL, UR, normal=n, riemann=O.ROE)
        F0 = O.point_flux(UL, UR, normal=n, riemann=O.ROE_NOFIX)
        assert np.array_equal(F, F0)
        up = UL if -S > 0 else UR
        ref = O.euler_normal_flux(up, n)
        assert np.max(np.abs(F - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_lax_friedrichs_structure():
    """Local Lax-Friedrichs: central flux minus a single scalar times the jump, the scalar
    being the larger of the two sides' spectral radii |v.n| + c."""
    rng = np.random.default_rng(12)
    for _ in range(30):
        UL, UR, n = rand_state(rng), rand_state(rng), rand_normal(rng)
        F = O.point_flux(UL, UR, normal=n, riemann=O.LF)
        FL, FR = O.euler_normal_flux(UL, n), O.euler_normal_flux(UR, n)
        lam = (FL + FR - 2.0 * F) / (UR - UL)
        assert np.max(np.abs(lam - lam[0])) < 1e-10 * lam[0]

        def radius(U):
            rho, v = U[0], U[1:4] / U[0]
            p = (GAMMA - 1.0) * (U[4] - 0.5 * rho * v @ v)
            return abs(v @ n) + math.sqrt(GAMMA * p / rho)
        assert abs(lam[0] - max(radius(UL), radius(UR))) < 1e-12


def test_roe_supersonic_is_full_upwind():
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = rand_normal(rng)
        UL = cons(1.0 + 0.01 * rng.uniform(), 2.5 * n + 0.01 * rng.normal(size=3), 0.71)
        UR = cons(1.0 + 0.01 * rng.uniform(), 2.5 * n + 0.01 * rng.normal(size=3), 0.72)
        F = O.point_flux(UL, UR, normal=n, riemann=O.ROE)
        assert np.max(np.abs(F - O.euler_normal_flux(UL, n))) < 1e-13
        # seen with the opposite normal the flow is supersonic towards the first state
        F = O.point_flux(UR, UL, normal=-n, riemann=O.ROE)
        assert np.max(np.abs(F - O.euler_normal_flux(UL, -n))) < 1e-13


def test_harten_hyman_fix_is_active_in_sonic_expansion_only():
    """The fix changes nothing unless an acoustic wave is a transonic expansion
    (lambda_L < 0 < lambda_R); there it adds dissipation, and it is continuous."""
    rng = np.random.default_rng(6)
    for _ in range(50):   # subsonic interface data of the workloads: fix inactive
        UL = cons(1 + 0.01 * rng.normal(), [0.3, 0, 0] + 0.01 * rng.normal(size=3), 0.71)
        UR = cons(1 + 0.01 * rng.normal(), [0.3, 0, 0] + 0.01 * rng.normal(size=3), 0.71)
        n = np.array([1.0, 0, 0])
        assert np.array_equal(O.point_flux(UL, UR, normal=n, riemann=O.ROE),
                              O.point_flux(UL, UR, normal=n, riemann=O.ROE_NOFIX))
    n = np.array([1.0, 0.0, 0.0])
    # sonic expansion in the u - c wave: u_L - c_L < 0 < u_R - c_R
    UL, UR = cons(1.0, [0.9, 0, 0], 1.0 / GAMMA), cons(0.8, [1.25, 0, 0], 0.75 / GAMMA)
    F = O.point_flux(UL, UR, normal=n, riemann=O.ROE)
    F0 = O.point_flux(UL, UR, normal=n, riemann=O.ROE_NOFIX)
    assert np.max(np.abs(F - F0)) > 1e-4
    # Harten's smooth form keeps the modulus continuously differentiable where the fix
    # switches on (|lambda~| = delta): second differences stay O(h^2) along a scan that
    # crosses the switch, while a kink would leave O(h)
    us = np.linspace(0.6, 1.2, 6001)          # h = 1e-4
    f = np.array([O.point_flux(cons(1.0, [u, 0, 0], 1.0 / GAMMA), UR, normal=n, riemann=O.ROE)
                  for u in us])
    fix_on = [not np.array_equal(fi, O.point_flux(cons(1.0, [u, 0, 0], 1.0 / GAMMA), UR,
                                                   normal=n, riemann=O.ROE_NOFIX))
              for u, fi in zip(us[::50], f[::50])]
    assert any(fix_on) and not all(fix_on)   # the scan crosses the switch
    assert np.max(np.abs(f[:-2] - 2 * f[1:-1] + f[2:])) < 1e-6


def test_viscous_linear_shear_and_heat_flux():
    mu, Pr = 1e-3, 0.72
    rng = np.random.default_rng(7)
    for _ in range(10):
        a, vy = rng.uniform(-1, 1), rng.uniform(-0.5, 0.5)
        U = cons(1.0, [0.0, vy, 0.0], 0.9)
        g = np.zeros((3, 5))
        g[0, 2] = a               # d(rho v)/dx with rho = 1:  dv/dx = a
        g[0, 4] = vy * a          # d(rho E)/dx keeps the pressure uniform
        Fv = O.viscous_normal_flux(U, g.ravel(), [1.0, 0.0, 0.0], GAMMA, mu, Pr)
        assert np.max(np.abs(Fv - [0, 0, mu * a, 0, mu * a * vy])) < 1e-17
        # pure pressure gradient at rest, uniform density: q = -mu gamma/((gamma-1)Pr) dp/dx / rho
        U = cons(1.3, [0.0, 0.0, 0.0], 0.9)
        g = np.zeros((3, 5))
        g[1, 4] = a / (GAMMA - 1.0)   # dp/dy = a
        Fv = O.viscous_normal_flux(U, g.ravel(), [0.0, 1.0, 0.0], GAMMA, mu, Pr)
        expect = mu * GAMMA / ((GAMMA - 1.0) * Pr) * a / 1.3
        assert np.max(np.abs(Fv - [0, 0, 0, 0, expect])) < 1e-16
        # uniform compression at rest: tau_xx = 2 mu a - 2/3 mu a (Stokes hypothesis)
        U = cons(1.0, [0.0, 0.0, 0.0], 0.9)
        g = np.zeros((3, 5))
        g[0, 1] = a               # du/dx = a, kinetic energy gradient vanishes at rest
        Fv = O.viscous_normal_flux(U, g.ravel(), [1.0, 0.0, 0.0], GAMMA, mu, Pr)
        assert np.max(np.abs(Fv - [0, 4.0 / 3.0 * mu * a, 0, 0, 0])) < 1e-17
        Fv = O.viscous_normal_flux(U, g.ravel(), [0.0, 1.0, 0.0], GAMMA, mu, Pr)
        assert np.max(np.abs(Fv - [0, 0, -2.0 / 3.0 * mu * a, 0, 0])) < 1e-17
        # density gradient at uniform pressure and velocity: no stress, heat flux from
        # dT = -p/rho^2 drho only
        vel = rng.uniform(-0.5, 0.5, 3)
        U = cons(1.3, vel, 0.9)
        g = np.zeros((3, 5))
        g[2, 0] = a
        g[2, 1:4] = vel * a
        g[2, 4] = 0.5 * (vel @ vel) * a
        Fv = O.viscous_normal_flux(U, g.ravel(), [0.0, 0.0, 1.0], GAMMA, mu, Pr)
        expect = -mu * GAMMA / ((GAMMA - 1.0) * Pr) * 0.9 / 1.3 ** 2 * a
        assert np.max(np.abs(Fv - [0, 0, 0, 0, expect])) < 1e-16
    U = rand_state(rng)
    assert np.all(O.viscous_normal_flux(U, np.zeros(15), rand_normal(rng)) == 0.0)


def test_br1_average_and_surface_element():
    rng = np.random.default_rng(8)
    for _ in range(10):
        UL, UR, n = rand_state(rng), rand_state(rng), rand_normal(rng)
        gL, gR = rng.normal(size=15) * 0.1, rng.normal(size=15) * 0.1
        F = O.point_flux(UL, UR, gL, gR, normal=n, dS=0.37, physics=O.NS, riemann=O.ROE, mu=1e-3)
        Fc = O.point_flux(UL, UR, normal=n, dS=1.0, physics=O.EULER, riemann=O.ROE)
        FvL = O.viscous_normal_flux(UL, gL, n, GAMMA, 1e-3, 0.72)
        FvR = O.viscous_normal_flux(UR, gR, n, GAMMA, 1e-3, 0.72)
        assert np.max(np.abs(F - 0.37 * (Fc - 0.5 * (FvL + FvR)))) < 1e-15

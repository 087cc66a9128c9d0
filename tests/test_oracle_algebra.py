"""Pins of the oracle's moment algebra against definitions the paper states.

Each expected value here is computed by a different route than the oracle
takes: raw/central moments straight from their definition (sums over the
D2Q9 velocity set, App. B), equilibria and sources from the continuous
Maxwellian plus lattice sums of the rest weights (App. C), the gradient
stencil from its exact Fourier symbol.
"""
import numpy as np
import pytest

# D2Q9 velocity set and weights, standard (App. B)
E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=float)
WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CS2 = 1.0 / 3.0
ORDERS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]


def raw_moments(f):
    return np.array([np.sum(f * E[:, 0] ** m * E[:, 1] ** n) for m, n in ORDERS])


def central_moments(f, ux, uy):
    return np.array([np.sum(f * (E[:, 0] - ux) ** m * (E[:, 1] - uy) ** n) for m, n in ORDERS])


def maxwell_central(rho):
    """Central moments of the continuous Maxwellian with density rho, c_s^2 = 1/3."""
    return np.array([rho, 0, 0, rho * CS2, rho * CS2, 0, 0, 0, rho * CS2 * CS2])


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def test_P_times_Pinv_is_identity(O):
    P, Pi = O.matrix_P(), O.matrix_Pinv()
    assert np.allclose(P @ Pi, np.eye(9), atol=1e-15)
    assert np.allclose(Pi @ P, np.eye(9), atol=1e-15)


def test_P_gives_raw_moments_by_definition(O):
    rng = np.random.default_rng(1)
    P = O.matrix_P()
    for _ in range(5):
        f = rng.normal(size=9)
        assert np.allclose(P @ f, raw_moments(f), atol=1e-13)


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.05, -0.02), (-0.13, 0.21), (0.3, 0.3)])
def test_F_gives_central_moments_by_definition(O, u):
    """Pins the last row of F (binomial reading): as printed it fails here."""
    rng = np.random.default_rng(2)
    P, F = O.matrix_P(), O.matrix_F(*u)
    for _ in range(5):
        f = rng.normal(size=9)
        assert np.allclose(F @ (P @ f), central_moments(f, *u), atol=1e-13)


@pytest.mark.parametrize("u", [(0.05, -0.02), (-0.13, 0.21)])
def test_Finv_is_inverse_and_F_of_minus_u(O, u):
    F, Fi = O.matrix_F(*u), O.matrix_Finv(*u)
    assert np.allclose(F @ Fi, np.eye(9), atol=1e-14)
    assert np.allclose(Fi, O.matrix_F(-u[0], -u[1]), atol=0)


@pytest.mark.parametrize("p,rho,ux,uy", [(1e-3, 1.0, 0.01, -0.02), (-2e-4, 0.1, -0.05, 0.03), (0.0, 0.55, 0.1, 0.0)])
def test_g_equilibrium_is_incompressible_transform(O, p, rho, ux, uy):
    """g_eq = c_s^2 f_M(rho, u) + (p - rho c_s^2) w  (He-Chen-Zhang transform):
    central moments = c_s^2 * Maxwellian central moments + varphi * lattice
    central moments of the rest weights."""
    vp = p - rho * CS2
    expected = CS2 * maxwell_central(rho) + vp * central_moments(WT, ux, uy)
    assert np.allclose(O.eq_g(p, rho, ux, uy), expected, rtol=1e-12, atol=1e-17)


@pytest.mark.parametrize("F", [(1e-5, -2e-5, 3e-6, 4e-6), (0.0, 1e-4, -2e-4, 0.0)])
@pytest.mark.parametrize("u", [(0.02, -0.01), (-0.1, 0.07)])
def test_g_source_is_central_moment_of_forcing(O, F, u):
    """Source S_a = (e_a - u).[Gamma_a(u) F_t + (Gamma_a(u) - Gamma_a(0)) F_p]:
    the Gamma(u) part is taken from the continuous Maxwellian (first moment
    c_s^2 delta, odd moments 0), the Gamma(0) part from lattice sums of w.
    Orders 0-2 must match; the paper sets 3rd/4th order to zero."""
    Ftx, Fty, Fpx, Fpy = F
    ux, uy = u
    expected = np.zeros(9)
    # Gamma(u) part: central moments of Gamma(u) (e - u) . F
    expected[1] = CS2 * (Ftx + Fpx)
    expected[2] = CS2 * (Fty + Fpy)
    # minus Gamma(0) part
    proj = (E[:, 0] - ux) * Fpx + (E[:, 1] - uy) * Fpy
    expected -= central_moments(WT * proj, ux, uy)
    got = O.source_g(Ftx, Fty, Fpx, Fpy, ux, uy)
    assert np.allclose(got[:6], expected[:6], rtol=1e-12, atol=1e-20)
    assert np.all(got[6:] == 0)


@pytest.mark.parametrize("omega1", [1.0, 1.25, 1.9])
def test_advection_diffusion_collision(O, omega1):
    """Post-collision central moments: zeroth conserved, first relaxed at
    omega1 toward (jx, jy), all higher moments at their equilibrium
    (X c_s^2, X c_s^2, 0, 0, 0, X c_s^4) (App. B, D, E)."""
    rng = np.random.default_rng(3)
    for _ in range(4):
        pop = WT * (0.3 + 0.05 * rng.normal(size=9))
        X = pop.sum()
        ux, uy = rng.uniform(-0.1, 0.1, size=2)
        jx, jy = rng.uniform(-1e-3, 1e-3, size=2)
        out = O.collide_ad(pop, X, jx, jy, omega1, ux, uy)
        k0 = central_moments(pop, ux, uy)
        k1 = central_moments(out, ux, uy)
        exp = np.array([X, k0[1] + omega1 * (jx - k0[1]), k0[2] + omega1 * (jy - k0[2]),
                        X * CS2, X * CS2, 0, 0, 0, X * CS2 * CS2])
        assert np.allclose(k1, exp, atol=1e-14)


@pytest.mark.parametrize("om", [1.0, 1.25, 0.6])
def test_two_fluid_collision(O, om):
    """Post-collision central moments of g (App. C) against equilibria and
    sources derived in this file (not the oracle's): rate-1 moments land on
    eq + sigma/2, the deviatoric pair (2d, 11) relaxes at omega_nu."""
    rng = np.random.default_rng(4)
    for _ in range(4):
        p, rho = 1e-4 * rng.normal(), rng.uniform(0.1, 1.0)
        ux, uy = rng.uniform(-0.05, 0.05, size=2)
        Ftx, Fty, Fpx, Fpy = 1e-5 * rng.normal(size=4)
        vp = p - rho * CS2
        eq = CS2 * maxwell_central(rho) + vp * central_moments(WT, ux, uy)
        proj = (E[:, 0] - ux) * Fpx + (E[:, 1] - uy) * Fpy
        src = -central_moments(WT * proj, ux, uy)
        src[1] += CS2 * (Ftx + Fpx)
        src[2] += CS2 * (Fty + Fpy)
        src[6:] = 0
        g = WT * p + 1e-5 * rng.normal(size=9)
        out = O.collide_g(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om)
        k0, k1 = central_moments(g, ux, uy), central_moments(out, ux, uy)
        for i in (0, 1, 2, 6, 7, 8):
            assert k1[i] == pytest.approx(eq[i] + 0.5 * src[i], abs=1e-16)
        assert k1[3] + k1[4] == pytest.approx(eq[3] + eq[4] + 0.5 * (src[3] + src[4]), abs=1e-16)
        d0, deq, dsrc = k0[3] - k0[4], eq[3] - eq[4], src[3] - src[4]
        assert k1[3] - k1[4] == pytest.approx(d0 + om * (deq - d0) + (1 - om / 2) * dsrc, abs=1e-16)
        assert k1[5] == pytest.approx(k0[5] + om * (eq[5] - k0[5]) + (1 - om / 2) * src[5], abs=1e-16)


@pytest.mark.parametrize("a,b", [(1, 0), (2, 3), (5, 1)])
def test_isotropic_gradient_symbol(O, a, b):
    """On X = sin(kx x + ky y) the stencil (1/cs2) sum w e X(x+e) returns
    exactly sin(kx)(2 + cos ky)/3 cos(...) for d/dx (its Fourier symbol)."""
    n = 32
    kx, ky = 2 * np.pi * a / n, 2 * np.pi * b / n
    y, x = np.mgrid[0:n, 0:n].astype(float)
    X = np.sin(kx * x + ky * y)
    gx, gy = O.grad_periodic(X)
    assert np.allclose(gx, np.sin(kx) * (2 + np.cos(ky)) / 3 * np.cos(kx * x + ky * y), atol=1e-14)
    assert np.allclose(gy, np.sin(ky) * (2 + np.cos(kx)) / 3 * np.cos(kx * x + ky * y), atol=1e-14)


def test_gradient_consistent_for_smooth_field(O):
    n = 128
    k = 2 * np.pi / n
    y, x = np.mgrid[0:n, 0:n].astype(float)
    gx, _ = O.grad_periodic(np.sin(k * x) * np.cos(k * y))
    assert np.allclose(gx, k * np.cos(k * x) * np.cos(k * y), atol=k * 2e-3)


def test_splitmix64_reference_outputs(O):
    """Published splitmix64 outputs for seed 1234567 (Vigna's reference)."""
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
           16408922859458223821]
    assert [O.splitmix64(1234567, k) for k in range(5)] == ref

"""Pins of the oracle's wall treatment (walls of Sec. 2; the paper is silent
on how finite differences and streaming meet a wall).

Readings pinned here:
  * walls sit at the half-link, x = -1/2 and nx - 1/2 (y likewise);
  * a finite-difference ghost takes its mirror node across that wall (zero
    normal gradient), or 2 X_w - X(mirror) on a Dirichlet wall, depth 2 for
    phi and depth 1 for T, psi, p*;
  * a streamed population whose source lies beyond a wall is bounced back
    (halfway) or anti-bounced back (Dirichlet T or psi), the y wall's rule
    applying on corner links.

Each expected value comes from a closed form or an analytic continuation of
a field that the stated wall condition extends exactly, never from the
oracle's own ghost code: a field even about x = -1/2 is its own mirror
extension, and a linear field is its own 2 X_w - X extension.  A
node-centred mirror, a dropped Dirichlet ghost or a ghost taken at the wrong
wall point each fails at least one test.
"""
import numpy as np
import pytest

from paper_2408_00146_amd import cases

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def iso_grad(X):
    """Isotropic gradient (Sec. 3) of the interior of an array padded by one
    node on every side: (1/cs2) sum_a w_a e_a X(x + e_a)."""
    ny, nx = X.shape[0] - 2, X.shape[1] - 2
    gx = np.zeros((ny, nx))
    gy = np.zeros((ny, nx))
    for a in range(1, 9):
        ex, ey = E[a]
        sh = X[1 + ey:1 + ey + ny, 1 + ex:1 + ex + nx]
        gx += 3.0 * WT[a] * ex * sh
        gy += 3.0 * WT[a] * ey * sh
    return gx, gy


def box(nx, ny, **kw):
    c = cases.periodic_box(8)
    c.update(nx=nx, ny=ny, **kw)
    return c


def slab_y(nx, ny, yc, R, W):
    """phi(y) of a flat slab |y - yc| < R with the tanh profile (Sec. 3): a
    function of y alone, so its x-derivatives vanish exactly."""
    y = np.arange(ny, dtype=float)[:, None]
    return np.broadcast_to(0.5 + 0.5 * np.tanh(2.0 * (R - np.abs(y - yc)) / W), (ny, nx)).copy()


def test_mirror_ghosts_sit_at_the_half_link(O):
    """phi = A + B cos(kx (x + 1/2)) + C cos(ky (y + 1/2)) with kx = pi/nx,
    ky = pi/ny is even about every wall at the half-link, so the mirror
    rule continues it exactly: the oracle's gradient at every node, the
    wall-adjacent ones included, equals the stencil of the analytic field,
    -B sin(kx) sin(kx (x + 1/2)) (y likewise), and the curvature (which
    reads phi two nodes beyond the wall) equals the isotropic divergence of
    the analytic normal.  A node-centred mirror gives 0 for the gradient at
    the wall-adjacent nodes instead."""
    nx, ny = 24, 16
    A, B, C = 0.5, 0.3, 0.2
    kx, ky = np.pi / nx, np.pi / ny
    c = box(nx, ny, wall=[1, 1, 1, 1], t_bc=[0, 0, 0, 0], psi_bc=[0, 0, 0, 0])
    o = O.Oracle(c)

    def phi_of(i, j):
        return A + B * np.cos(kx * (i + 0.5)) + C * np.cos(ky * (j + 0.5))

    x, y = np.meshgrid(np.arange(nx, dtype=float), np.arange(ny, dtype=float))
    o.load_fields(phi_of(x, y), 0.5, 0.0)
    it = o.intermediates()
    gx_cf = -B * np.sin(kx) * np.sin(kx * (x + 0.5))
    gy_cf = -C * np.sin(ky) * np.sin(ky * (y + 0.5))
    assert np.max(np.abs(it["dphi_dx"] - gx_cf)) <= 1e-15
    assert np.max(np.abs(it["dphi_dy"] - gy_cf)) <= 1e-15
    # the pin has teeth: the wall-adjacent gradient is far from a node-centred mirror's 0
    assert np.min(np.abs(gx_cf[:, 0])) > 1e-3 and np.min(np.abs(gy_cf[0, :])) > 1e-3

    # curvature from the analytic field two nodes beyond every wall
    xe, ye = np.meshgrid(np.arange(-2, nx + 2, dtype=float), np.arange(-2, ny + 2, dtype=float))
    gxe, gye = iso_grad(phi_of(xe, ye))  # gradient on nodes -1 .. n
    mag = np.maximum(np.hypot(gxe, gye), 1e-12)
    nxe, nye = gxe / mag, gye / mag
    kap = iso_grad(nxe)[0] + iso_grad(nye)[1]
    assert np.max(np.abs(it["kappa"] - kap)) <= 1e-13 * np.max(np.abs(kap))


@pytest.mark.parametrize("walls", ["x_dirichlet", "all_dirichlet"])
def test_dirichlet_temperature_ghost_extends_linear_T(O, walls):
    """A linear wall law T_w(x) = T0 + G (x - xT0) held on Dirichlet walls,
    with T = T_w(x) everywhere: 2 T_w - T(mirror), taken at the wall point,
    continues a linear T exactly (at corners too), so with sigma linear in T
    the tangential CSF force on a flat slab, 1.5 W |grad phi|^2 d(sigma)/dx
    (Sec. 3), equals 1.5 W |grad phi|^2 sigma_T G at every node.  Without
    the Dirichlet ghost (plain mirror) the wall-adjacent value halves."""
    nx, ny, W, G, sT = 20, 24, 4.0, 0.02, -3e-4
    if walls == "x_dirichlet":
        c = box(nx, ny, wall=[1, 1, 0, 0], t_bc=[1, 1, 0, 0])
    else:
        c = box(nx, ny, wall=[1, 1, 1, 1], t_bc=[1, 1, 1, 1])
    c.update(T0=0.5, gradT=G, xT0=7.3, sigma_law=cases.SIGMA_MULT, sigma0=1e-3, sigma_T=sT, sigma_TT=0.0,
             T_ref=0.5, beta_s=0.0, W=W)
    o = O.Oracle(c)
    phi = slab_y(nx, ny, ny / 2.0, ny / 4.0, W)
    T = 0.5 + G * (np.arange(nx, dtype=float) - 7.3)[None, :] * np.ones((ny, 1))
    o.load_fields(phi, T, 0.0)
    it = o.intermediates()
    assert np.max(np.abs(it["dphi_dx"])) == 0.0
    g2 = it["dphi_dx"] ** 2 + it["dphi_dy"] ** 2
    expect = 1.5 * W * g2 * sT * G
    assert np.max(np.abs(it["Fs_x"] - expect)) <= 1e-12 * np.max(np.abs(expect))
    assert np.max(np.abs(expect[:, 0])) > 0.1 * np.max(np.abs(expect))


@pytest.mark.parametrize("axis", ["x", "y"])
def test_dirichlet_psi_ghost_extends_linear_psi(O, axis):
    """Dirichlet psi walls (Sec. 2: psi_L, psi_R) with psi linear between
    them, psi = psi_w at the half-link wall points: the ghost 2 psi_w -
    psi(mirror) continues it exactly, so the Marangoni part of the CSF force
    along the wall-normal axis, across a flat interface parallel to it,
    equals 1.5 W |grad phi|^2 (sigma(psi(i+1)) - sigma(psi(i-1))) / 2 with
    sigma from the continued linear psi (Langmuir factor, Sec. 2.1)."""
    n_w, n_t, W = 20, 24, 4.0  # nodes across the walls, nodes along them
    s0, beta, pw0, pw1 = 1e-3, 0.3, 0.45, 0.05
    if axis == "x":
        nx, ny = n_w, n_t
        c = box(nx, ny, wall=[1, 1, 0, 0], psi_bc=[1, 1, 0, 0], psi_w=[pw0, pw1, 0.0, 0.0])
    else:
        nx, ny = n_t, n_w
        c = box(nx, ny, wall=[0, 0, 1, 1], psi_bc=[0, 0, 1, 1], psi_w=[0.0, 0.0, pw0, pw1])
    c.update(sigma_law=cases.SIGMA_MULT, sigma0=s0, sigma_T=0.0, sigma_TT=0.0, beta_s=beta, psi_inf=1.0,
             W=W, gradT=0.0)
    o = O.Oracle(c)
    s = np.arange(-1, n_w + 1, dtype=float)
    psi_line = pw0 + (pw1 - pw0) * (s + 0.5) / n_w
    sig = s0 * (1.0 + beta * np.log(1.0 - psi_line))
    dsig = 0.5 * (sig[2:] - sig[:-2])
    if axis == "x":
        phi = slab_y(nx, ny, ny / 2.0, ny / 4.0, W)
        psi = np.broadcast_to(psi_line[1:-1][None, :], (ny, nx)).copy()
        ds = np.broadcast_to(dsig[None, :], (ny, nx))
    else:
        phi = slab_y(ny, nx, nx / 2.0, nx / 4.0, W).T.copy()
        psi = np.broadcast_to(psi_line[1:-1][:, None], (ny, nx)).copy()
        ds = np.broadcast_to(dsig[:, None], (ny, nx))
    o.load_fields(phi, 0.5, psi)
    it = o.intermediates()
    g2 = it["dphi_dx"] ** 2 + it["dphi_dy"] ** 2
    F = it["Fs_x"] if axis == "x" else it["Fs_y"]
    expect = 1.5 * W * g2 * ds
    assert np.max(np.abs(F - expect)) <= 1e-12 * np.max(np.abs(expect))


@pytest.mark.parametrize("law", [cases.SIGMA_MULT, cases.SIGMA_PAPER])
def test_sigma_law_temperature_surfactant_coupling(O, law):
    """Sec. 2.1: the printed law's surfactant term carries the factor T/T_ref,
    so d2 sigma/dT dpsi at (T_ref, 0) is -beta sigma0 / T_ref and the
    Langmuir slope d sigma/d psi at psi = 0 doubles when T doubles; in the
    multiplicative variant d2 sigma/dT dpsi = -beta sigma_T / psi_inf and the
    slope at T = 2 T_ref is -beta (sigma0 + sigma_T T_ref + sigma_TT T_ref^2)
    / psi_inf.  Dropping T/T_ref from the printed law fails both."""
    s0, sT, sTT, Tr, beta = 2e-3, -3e-4, 5e-4, 0.7, 0.25
    c = cases.periodic_box(8)
    c.update(sigma_law=law, sigma0=s0, sigma_T=sT, sigma_TT=sTT, T_ref=Tr, beta_s=beta, psi_inf=1.0)
    o = O.Oracle(c)

    def sig(T, psi):
        o.load_fields(0.0, T, psi)
        return o.intermediates()["sigma"][3, 3]

    h = 1e-4
    mixed = (sig(Tr + h, h) - sig(Tr + h, -h) - sig(Tr - h, h) + sig(Tr - h, -h)) / (4 * h * h)
    want = -beta * s0 / Tr if law == cases.SIGMA_PAPER else -beta * sT
    assert mixed == pytest.approx(want, rel=1e-6)
    hp = 1e-7
    slope2 = (sig(2 * Tr, hp) - sig(2 * Tr, -hp)) / (2 * hp)
    if law == cases.SIGMA_PAPER:
        want2 = -beta * s0 * 2.0
    else:
        want2 = -beta * (s0 + sT * Tr + sTT * Tr * Tr)
    assert slope2 == pytest.approx(want2, rel=1e-6)


@pytest.mark.parametrize("periodic_x", [False, True])
def test_streaming_links_by_brute_force(O, periodic_x):
    """Every streamed population of a 5x4 lattice from random post-collision
    values, against a per-link enumeration of the rules: a source inside the
    lattice (after periodic wrap) is pulled; beyond one wall the link bounces
    back, X_a(x) = X~_abar(x), or for a Dirichlet T / psi wall anti-bounces
    back, -X~_abar(x) + 2 w_a X_w with T_w at the link midpoint x - e_a/2;
    beyond an x wall and a y wall at once (corner links) the y wall's rule
    applies.  The x walls carry Dirichlet T and the y walls Dirichlet psi, so
    a corner link taking the x wall's rule fails for both sets."""
    nx, ny = 5, 4
    G, T0, xT0 = 0.07, 0.4, 1.5
    pw = [0.0, 0.0, 0.31, 0.17]
    if periodic_x:
        c = box(nx, ny, wall=[0, 0, 1, 1], t_bc=[0, 0, 1, 1], psi_bc=[0, 0, 1, 1], psi_w=pw)
    else:
        c = box(nx, ny, wall=[1, 1, 1, 1], t_bc=[1, 1, 0, 0], psi_bc=[0, 0, 1, 1], psi_w=pw)
    c.update(T0=T0, gradT=G, xT0=xT0)
    o = O.Oracle(c)
    rng = np.random.default_rng(11)
    post = rng.normal(size=(4, 9, ny, nx))
    got = o.stream_only(post)
    wx, wy = c["wall"][0] == 1, c["wall"][2] == 1
    for j in range(ny):
        for i in range(nx):
            for a in range(9):
                si, sj = i - E[a][0], j - E[a][1]
                if not wx:
                    si %= nx
                outx, outy = not (0 <= si < nx), not (0 <= sj < ny)
                if not outx and not outy:
                    want = post[:, a, sj, si]
                else:
                    side = (2 if sj < 0 else 3) if outy else (0 if si < 0 else 1)
                    b = OPP[a]
                    want = post[:, b, j, i].copy()
                    if c["t_bc"][side]:
                        Tw = T0 + G * (i - 0.5 * E[a][0] - xT0)
                        want[2] = -post[2, b, j, i] + 2 * WT[a] * Tw
                    if c["psi_bc"][side]:
                        want[3] = -post[3, b, j, i] + 2 * WT[a] * pw[side]
                assert np.allclose(got[:, a, j, i], want, rtol=0, atol=1e-15), (i, j, a)

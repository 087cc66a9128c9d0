"""Seeded synthetic workloads in lattice units.

This module only chooses parameters (grid, walls, property values, the
random draws of the batched sweeps).  It contains none of the method's
arithmetic and imports nothing from the GPU library or the oracle, so both
the GPU binding and the oracle can be driven from the same case dicts.

Every workload is a synthetic channel shaped like the paper's (aspect 2:1,
bubble in the upstream half, Sec. 2); the paper uses no dataset.
"""
from __future__ import annotations

import math

import numpy as np

FP64, FP32, FP16S = 0, 1, 2
SIGMA_MULT, SIGMA_PAPER = 0, 1
INIT_BUBBLE, INIT_SLAB, INIT_NONE = 0, 1, 2

# Surfactant groups of Sec. 6 (Pi = lambda W^2 / (8 sigma0), Ex = 4 s / (w W^2)).
PI_RESULTS, EX_RESULTS = 8.33, 0.16


def surfactant_ratios(W: float, Pi: float, Ex: float) -> tuple[float, float]:
    """(s/lambda, w/lambda) from the groups Pi and Ex.

    Two groups cannot fix three parameters; the reading taken is s = 8 sigma0,
    which makes Pi = s-normalised diffusion strength.  Then
    s/lambda = W^2 / Pi and w/lambda = 4 / (Ex Pi)."""
    return W * W / Pi, 4.0 / (Ex * Pi)


def base(**kw) -> dict:
    """Defaults shared by all channel workloads; override with keywords."""
    W = kw.get("W", 4.0)
    s_lam, w_lam = surfactant_ratios(W, PI_RESULTS, EX_RESULTS)
    c = dict(
        nx=128, ny=64, precision=FP64, sigma_law=SIGMA_MULT, init_kind=INIT_BUBBLE,
        wall=[1, 1, 1, 1], t_bc=[0, 0, 1, 1], psi_bc=[0, 0, 0, 0], psi_w=[0.0, 0.0, 0.0, 0.0],
        T0=0.5, gradT=0.01, xT0=64.0,
        sigma0=1e-3, sigma_T=0.0, sigma_TT=1e-4, T_ref=0.5, beta_s=0.1, psi_inf=1.0,
        rho_A=1.0, rho_B=0.1, nu_A=0.1, nu_B=0.1, alpha_A=0.05, alpha_B=0.05,
        D_psi=0.01, M_phi=0.1, W=W, s_lam=s_lam, w_lam=w_lam,
        Fext_x=0.0, Fext_y=0.0, gravity=0.0,
        xc=40.0, yc=32.0, R=10.0, psi_bulk=0.0, psi_band=0.1, phi_noise=1e-6, p_jump=0.0, psi_gradx=0.0, seed=0,
        max_steps=0,
    )
    c.update(kw)
    return c


def channel(nx: int, ny: int, R: float, W: float, *, dT: float = None, gradT: float = None, **kw) -> dict:
    """SRF channel: walls all round, Dirichlet T_w(x) = T0 + G (x - nx/2) on the
    top/bottom walls, zero-flux x ends, bubble of radius R at (nx/4, ny/2).
    G defaults to dT / nx with dT = 1.28 (the temperature span of the small
    FP64 channel, 0.01 x 128)."""
    if gradT is None:
        gradT = (1.28 if dT is None else dT) / nx
    return base(nx=nx, ny=ny, R=float(R), W=float(W), xc=nx / 4.0, yc=ny / 2.0,
                gradT=gradT, xT0=nx / 2.0, **kw)


# ------------------------------------------------------------------ workloads

def config_small_fp64() -> dict:
    """128x64 plain method in FP64: R = 10 at (40, 32), W = 4, density ratio 10,
    nu = 0.1, alpha = 0.05, D_psi = 0.01, T_w = T0 + 0.01 (x - 64), SRF law
    1e-3 + 1e-4 (T - T0)^2 times (1 + 0.1 ln(1 - psi)); 2000 steps."""
    return base()


def marangoni_gradient(kind: str, nx: int, R: float, mu_A: float, alpha: float, sigma_T: float,
                       sigma_TT: float, Ma: float) -> float:
    """Wall-temperature gradient G giving Marangoni number Ma = U_o R / alpha_A
    with the paper's thermocapillary velocity U_o = (sigma0/mu_A)(R/L)(M1 + M2)
    (Sec. 6) and L = nx, dT = G L: NF U_o = |sigma_T| G R / mu_A;
    SRF U_o = sigma_TT G^2 L R / mu_A."""
    if kind == "NF":
        return Ma * mu_A * alpha / (abs(sigma_T) * R * R)
    return math.sqrt(Ma * mu_A * alpha / (sigma_TT * nx * R * R))


def config_fp32_runs() -> list[dict]:
    """1024x512, R = 80 at (256, 256), W = 5; NF (sigma_T = -1e-5) and SRF
    (sigma_TT = 1e-4) at beta_s in {0, 0.2}; gradient set for Ma = 10."""
    out = []
    for kind in ("NF", "SRF"):
        for beta in (0.0, 0.2):
            sT, sTT = (-1e-5, 0.0) if kind == "NF" else (0.0, 1e-4)
            G = marangoni_gradient(kind, 1024, 80.0, 0.1, 0.05, sT, sTT, 10.0)
            c = channel(1024, 512, 80.0, 5.0, gradT=G, precision=FP32, sigma_T=sT, sigma_TT=sTT, beta_s=beta)
            c["xc"], c["yc"] = 256.0, 256.0
            c["label"] = f"{kind}-beta{beta}"
            out.append(c)
    return out


def config_precision(precision: int = FP16S) -> dict:
    """2048x1024, R = 128 at (512, 512), W = 5, ratio 10, sigma_TT = 1e-4, beta_s = 0.3."""
    c = channel(2048, 1024, 128.0, 5.0, precision=precision, sigma_TT=1e-4, beta_s=0.3)
    c["xc"], c["yc"] = 512.0, 512.0
    return c


def sweep_cases(n: int, seed: int, sizes=(256, 384, 512, 768, 1024), precision: int = FP32,
                max_steps: int = 0) -> list[dict]:
    """n uneven channels drawn from numpy default_rng(seed): Nx uniform over
    `sizes`, Ny = Nx/2, R = Ny/6, W = 5, beta_s ~ U[0, 0.5],
    sigma_TT ~ logU[1e-5, 1e-3]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nx = int(rng.choice(np.asarray(sizes)))
        beta = float(rng.uniform(0.0, 0.5))
        sTT = float(10.0 ** rng.uniform(-5.0, -3.0))
        ny = nx // 2
        c = channel(nx, ny, ny / 6.0, 5.0, precision=precision, sigma_TT=sTT, beta_s=beta,
                    seed=seed * 100003 + k, max_steps=max_steps)
        c["label"] = f"sweep{seed}-{k}"
        out.append(c)
    return out


def config_batched() -> list[dict]:
    """64 uneven channels (seed 3), FP32, 5000 steps each."""
    return sweep_cases(64, 3, max_steps=5000)


def config_large_plus_small() -> list[dict]:
    """One 4096x2048 SRF channel (R = 256, W = 6, beta_s = 0.2, sigma_TT = 1e-4,
    FP16 storage, 5000 steps) plus 256 channels of 128x64 drawn as the sweep
    (seed 4), FP32, 2000 steps."""
    big = channel(4096, 2048, 256.0, 6.0, precision=FP16S, sigma_TT=1e-4, beta_s=0.2, max_steps=5000)
    big["xc"], big["yc"] = 1024.0, 1024.0
    big["label"] = "large"
    small = sweep_cases(256, 4, sizes=(128,), precision=FP32, max_steps=2000)
    return [big] + small


# ------------------------------------------------------- validation problems

def static_bubble(n: int = 64, R: float = 12.0, sigma: float = 1e-3, rho_ratio: float = 10.0,
                  W: float = 4.0, precision: int = FP64) -> dict:
    """Static bubble in a periodic box, constant sigma (Laplace law, Sec. 5)."""
    return base(nx=n, ny=n, precision=precision, wall=[0, 0, 0, 0], t_bc=[0, 0, 0, 0],
                sigma0=sigma, sigma_T=0.0, sigma_TT=0.0, beta_s=0.0, rho_A=1.0, rho_B=1.0 / rho_ratio,
                W=W, xc=n / 2.0, yc=n / 2.0, R=R, gradT=0.0, psi_band=0.0, phi_noise=0.0)


def laplace_hdr(n: int = 200, R: float = 25.0, sigma: float = 1e-3, precision: int = FP64) -> dict:
    """Static bubble at density ratio 1000 and viscosity ratio 100 in a
    periodic box (the Laplace test of Sec. 5.1), started at its Laplace
    pressure (from p = 0, or from a pressure step p_jump * phi0, a bubble of
    radius 20 at sigma = 4e-3 diverges within 50 steps)."""
    p = static_bubble(n=n, R=R, sigma=sigma, rho_ratio=1000.0, W=5.0, precision=precision)
    p.update(nu_A=0.1, nu_B=1.0, p_jump=sigma / R)
    return p


def poiseuille(ny: int = 32, nx: int = 4, F: float = 1e-6, nu: float = 0.5) -> dict:
    """Single-phase channel between no-slip walls at y = -1/2 and ny - 1/2,
    periodic in x, driven by a constant body force."""
    return base(nx=nx, ny=ny, wall=[0, 0, 1, 1], t_bc=[0, 0, 0, 0], init_kind=INIT_NONE,
                nu_A=nu, nu_B=nu, Fext_x=F, gradT=0.0, psi_band=0.0, phi_noise=0.0, beta_s=0.0)


def periodic_box(n: int = 64, alpha: float = 0.05, D_psi: float = 0.01) -> dict:
    """Single fluid at rest in a periodic box (scalar transport tests)."""
    return base(nx=n, ny=n, wall=[0, 0, 0, 0], t_bc=[0, 0, 0, 0], init_kind=INIT_NONE,
                alpha_A=alpha, alpha_B=alpha, D_psi=D_psi, gradT=0.0, psi_band=0.0, phi_noise=0.0,
                beta_s=0.0, s_lam=0.0, w_lam=0.0)


def conduction(nx: int = 32, ny: int = 4, alpha: float = 0.5, T_left: float = 1.0, T_right: float = 0.0) -> dict:
    """Dirichlet walls at x = -1/2 (T_left) and nx - 1/2 (T_right), periodic y."""
    G = (T_right - T_left) / nx
    return base(nx=nx, ny=ny, wall=[1, 1, 0, 0], t_bc=[1, 1, 0, 0], init_kind=INIT_NONE,
                alpha_A=alpha, alpha_B=alpha, T0=T_left + G * 0.5, gradT=G, xT0=0.0,
                psi_band=0.0, phi_noise=0.0, beta_s=0.0)


def flat_surfactant(psi_b: float, ny: int = 64, nx: int = 4) -> dict:
    """Flat interfaces (slab of half-width ny/4, periodic box) with the surfactant
    parameters of the paper's flat-interface test: W = 5, Ex = 0.025, Pi = 50,
    sigma0 = 0.01, M_phi = M_psi = 0.02 (Sec. 5)."""
    s_lam, w_lam = surfactant_ratios(5.0, 50.0, 0.025)
    return base(nx=nx, ny=ny, wall=[0, 0, 0, 0], t_bc=[0, 0, 0, 0], init_kind=INIT_SLAB,
                W=5.0, s_lam=s_lam, w_lam=w_lam, sigma0=0.01, sigma_TT=0.0, beta_s=0.0,
                M_phi=0.02, D_psi=0.02, xc=0.0, yc=ny / 2.0, R=ny / 4.0, gradT=0.0,
                psi_bulk=psi_b, psi_band=0.0, phi_noise=0.0)


def thermocapillary_nf(nx: int = 192, ny: int = 96, R: float = 12.0, G: float = 2e-3,
                       sigma_T: float = -1e-4, nu: float = 0.5, alpha: float = 0.5) -> dict:
    """Normal-fluid bubble in a linear temperature field (Young-Goldstein-Block
    drift): linear sigma(T), no surfactant effect, centred bubble."""
    return base(nx=nx, ny=ny, R=R, W=4.0, xc=nx / 2.0, yc=ny / 2.0, gradT=G, xT0=nx / 2.0,
                sigma0=1e-3, sigma_T=sigma_T, sigma_TT=0.0, beta_s=0.0, nu_A=nu, nu_B=nu,
                alpha_A=alpha, alpha_B=alpha, psi_band=0.0, phi_noise=0.0)


# ------------------------------------------------- the paper's migration problem

def srf_channel(M1: float = 0.0, M2: float = 5.0, beta: float = 0.0, psi_L: float = 0.4, psi_R: float = 0.1,
                L: int = 600, D_over_H: float = 0.1, x0_over_L: float = 0.25, Re: float = 5.0, Ma: float = 0.25,
                rho_ratio: float = 1000.0, mu_ratio: float = 100.0, sigma0: float = 5e-3, W: float = 5.0,
                M_phi: float = 0.1, M_psi: float = 0.01, Pi: float = 8.33, Ex: float = 0.16,
                precision: int = FP32, Uo: float = None) -> dict:
    """The surfactant-laden bubble migration problem of Sec. 2 and Sec. 6 from
    its dimensionless groups, in lattice units.

    Domain L x H with H = L/2; no-slip walls at x = -1/2 (hot, T_H = 1, psi_L)
    and x = L - 1/2 (cold, T_C = 0, psi_R), periodic in y; T and psi start
    linear between the walls, T_ref = 0.5 at mid-channel.  Bubble of diameter
    D = D_over_H H at (x0_over_L L, H/2), started at the Laplace pressure
    sigma0/R of the reference surface tension.  Printed (additive) sigma law with
    sigma_T = M1 sigma0 / dT and sigma_TT = M2 sigma0 / dT^2 (dT = 1).
    Velocity scale U_o = (sigma0/mu_A)(R/L)|M1 + M2| (Sec. 6); Re = U_o R/nu_A
    and Ma = U_o R/alpha_A (Sec. 2.1) fix nu_A and alpha_A (rho_A = 1);
    rho_B = rho_A/rho_ratio, mu_B = mu_A/mu_ratio, alpha_B = alpha_A.
    Surfactant chemical potential from Pi and Ex; D_psi = M_psi.

    Uo, if given, replaces sigma0 by the value that makes the velocity scale
    Uo (U_o^2 = sigma0 Re |M1 + M2| / L), every group unchanged: the light
    phase of the pressure-based scheme is compressed by about
    rho_A U_o^2 / (rho_B cs^2), so U_o must stay well below 0.3 / rho_ratio
    (2.5e-4 at the paper's density ratio of 1000)."""
    H = L // 2
    R = 0.5 * D_over_H * H
    dT = 1.0
    if Uo is not None:
        sigma0 = Uo * Uo * L / (Re * abs(M1 + M2))
    sT, sTT = M1 * sigma0 / dT, M2 * sigma0 / dT ** 2
    # U_o mu_A is fixed by sigma0, R/L, M1 + M2; Re then fixes mu_A = nu_A (rho_A = 1)
    Uo_muA = sigma0 * (R / L) * abs(M1 + M2)
    nu_A = (Uo_muA * R / Re) ** 0.5
    Uo = Uo_muA / nu_A
    alpha = Uo * R / Ma
    rho_B = 1.0 / rho_ratio
    nu_B = nu_A / mu_ratio / rho_B
    T_of = lambda x: 1.0 - (x + 0.5) / L
    xb, yb = x0_over_L * L - 0.5, 0.5 * H - 0.5
    s_lam, w_lam = surfactant_ratios(W, Pi, Ex)
    return base(nx=L, ny=H, precision=precision, wall=[1, 1, 0, 0], t_bc=[1, 1, 0, 0], psi_bc=[1, 1, 0, 0],
                psi_w=[psi_L, psi_R, 0.0, 0.0], T0=T_of(0.0), gradT=-dT / L, xT0=0.0,
                sigma_law=SIGMA_PAPER, sigma0=sigma0, sigma_T=sT, sigma_TT=sTT, T_ref=0.5, beta_s=beta,
                psi_inf=1.0, rho_A=1.0, rho_B=rho_B, nu_A=nu_A, nu_B=nu_B, alpha_A=alpha, alpha_B=alpha,
                D_psi=M_psi, M_phi=M_phi, W=W, s_lam=s_lam, w_lam=w_lam, xc=xb, yc=yb, R=R,
                psi_bulk=psi_L + (psi_R - psi_L) * 0.5 / L, psi_gradx=(psi_R - psi_L) / L, psi_band=0.0,
                phi_noise=0.0, p_jump=sigma0 / R)


def srf_scales(p: dict) -> dict:
    """Velocity and time scales of an srf_channel case: U_o and T_o = R/U_o."""
    M12 = abs(p["sigma_T"] + p["sigma_TT"]) / p["sigma0"]
    Uo = p["sigma0"] / (p["rho_A"] * p["nu_A"]) * (p["R"] / p["nx"]) * M12
    return {"Uo": Uo, "To": p["R"] / Uo}


# ------------------------------------------------- buoyancy-driven rising bubble

def rising_bubble(Eo: float, Re: float = 35.0, D: float = 80.0, nx: int = 161, ny: int = 481,
                  yc: float = 120.0, U0: float = 0.01, rho_ratio: float = 1000.0, mu_ratio: float = 100.0,
                  W: float = 5.0, M_phi: float = 0.1, precision: int = FP32) -> dict:
    """The rising bubble of Sec. 5.3 from its groups, in lattice units:
    nx x ny lattice, periodic in x, no-slip walls at the bottom and top, a
    bubble of diameter D centred at ((nx - 1)/2, yc), buoyancy
    F_y = -(rho - rho_A) g.  Gravitational velocity U0 = sqrt(g D) (chosen),
    Re = rho_A U0 D / mu_A and Eo = rho_A U0^2 D / sigma fix mu_A and sigma;
    rho_B = rho_A / rho_ratio, mu_B = mu_A / mu_ratio.  Time scale D / U0.
    The light phase of the pressure-based scheme is compressed by about
    rho_A U0^2 / (rho_B cs^2), so U0 must stay well below 0.3 / rho_ratio
    for phi to stay near 1 inside the bubble.
    The bubble starts at its Laplace pressure sigma / R; T and psi play no
    part (uniform T, no surfactant)."""
    g = U0 * U0 / D
    mu_A = U0 * D / Re  # rho_A = 1
    sigma = U0 * U0 * D / Eo
    rho_B = 1.0 / rho_ratio
    nu_B = mu_A / mu_ratio / rho_B
    return base(nx=nx, ny=ny, precision=precision, wall=[0, 0, 1, 1], t_bc=[0, 0, 0, 0], psi_bc=[0, 0, 0, 0],
                gradT=0.0, sigma_law=SIGMA_MULT, sigma0=sigma, sigma_T=0.0, sigma_TT=0.0, beta_s=0.0,
                rho_A=1.0, rho_B=rho_B, nu_A=mu_A, nu_B=nu_B, alpha_A=0.05, alpha_B=0.05, W=W, M_phi=M_phi,
                gravity=g, xc=(nx - 1) / 2.0, yc=yc, R=D / 2.0, psi_band=0.0, psi_bulk=0.0, phi_noise=0.0,
                p_jump=sigma / (D / 2.0), s_lam=0.0, w_lam=0.0)

"""Seeded synthetic workloads: parameter sets and initial fields.

This module is shared by the HIP path's tests and benchmark and by the CPU
oracle's tests.  It holds no step of the lattice Boltzmann method: only
parameter values (lattice units, dx = dt = 1, Sec. 4 preamble), initial
macroscopic fields (phi, u, T) and, for single-step parity tests, random
population arrays.  Both implementations build their own populations from
these fields.

The paper's experiments are initial-value problems, not datasets.  The sets
below stand in for them with the same structure: tanh interfaces between the
bulk values -1 and +1, cosine or linear wall temperatures, small velocities.

Boundary kinds per side (x-lo, x-hi, y-lo, y-hi):
PERIODIC, WALL_T (no-slip, Dirichlet T), WALL_ADIABATIC (no-slip, zero heat
flux), INLET (fully developed inflow, fixed phi and T), OUTLET (zero gradient).
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC, WALL_T, WALL_ADIABATIC, INLET, OUTLET = 0, 1, 2, 3, 4
XLO, XHI, YLO, YHI = 0, 1, 2, 3


def base_params(nx: int, ny: int) -> dict:
    """Defaults shared by every set: W = 3 (Sec. 4 preamble), mobility 0.1."""
    return dict(
        nx=int(nx), ny=int(ny), bc=[PERIODIC, PERIODIC, WALL_T, WALL_T], grad_mode=0,
        rho_l=1.0, rho_h=1.0, mu_l=0.1, mu_h=0.1, lambda_l=0.1, lambda_h=0.1, rhocp_l=1.0, rhocp_h=1.0,
        sigma_ref=1e-3, sigma_T=0.0, sigma_TT=0.0, T_ref=0.0, W=3.0, mobility=0.1, Gx=0.0, Gy=0.0,
        tw_mean=[0.0] * 4, tw_amp=[0.0] * 4, tw_k=[0.0] * 4, tw_slope=[0.0] * 4,
        u_in_mean=0.0, phi_in=1.0, T_in=0.0, phi0_dev=0.0, T0_dev=0.0,
        bubbles_x=[], bubbles_y=[], collision=0, trt_magic=3.0 / 16.0,
    )


def body_force_channel(ny: int = 32, mu: float = 0.5, G: float = 1e-6, collision: int = 0,
                       trt_magic: float = 3.0 / 16.0, nx: int = 4) -> tuple[dict, dict]:
    """One fluid (phi = 1 everywhere) between adiabatic no-slip walls at
    j = -1/2 and ny - 1/2, periodic in x, driven by the body force G along x:
    plane Poiseuille flow, u_x = G (y + 1/2)(ny - 1/2 - y) / (2 mu) at steady state."""
    p = base_params(nx, ny)
    p.update(bc=[PERIODIC, PERIODIC, WALL_ADIABATIC, WALL_ADIABATIC], mu_l=mu, mu_h=mu, Gx=G,
             collision=collision, trt_magic=trt_magic)
    phi = np.ones((ny, nx))
    return p, dict(phi=phi, ux=np.zeros_like(phi), uy=np.zeros_like(phi), T=np.zeros_like(phi))


def tanh_profile(d: np.ndarray, W: float) -> np.ndarray:
    """Equilibrium order-parameter profile tanh(d / (sqrt(2) W)), d the signed
    distance from the interface (positive on the heavy side)."""
    return np.tanh(d / (math.sqrt(2.0) * W))


def grid(nx: int, ny: int):
    j, i = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    return i, j


# ---------------------------------------------------------------------------
# Heated microchannel with two superimposed planar fluids (Sec. 4.1)
# ---------------------------------------------------------------------------

def heated_channel(lambda_ratio: float = 1.0, nx: int = 64, ny: int = 32, W: float = 4.0,
                   T0: float = 40.0, dT: float = 4.0) -> tuple[dict, dict]:
    """Heavy fluid (phi=+1) in y < ny/2, light fluid above; walls at
    j = -1/2 and ny - 1/2; bottom wall T0 + dT cos(2 pi x / nx), top wall T0.
    lambda_ratio = lambda_l / lambda_h.

    The unit normal of the Allen-Cahn source is taken from the stencil
    (grad_mode 1): at W = 4 in a 32-node channel the walls truncate the tanh
    tails, and where |grad phi| < (1 - 1/(2 tau_phi)) (1 - phi^2)/(sqrt2 W) the
    normal recovered from the moments points the wrong way; that region seeds a
    slowly growing mode that breaks the x -> -x symmetry."""
    p = base_params(nx, ny)
    p.update(bc=[PERIODIC, PERIODIC, WALL_T, WALL_T], W=W, grad_mode=1,
             rho_l=1.0, rho_h=1.0, mu_l=0.2, mu_h=0.2, rhocp_l=1.0, rhocp_h=1.0,
             lambda_h=0.2, lambda_l=0.2 * lambda_ratio,
             sigma_ref=2.5e-2, sigma_T=-5e-4, sigma_TT=0.0, T_ref=T0)
    p["tw_mean"] = [0.0, 0.0, T0, T0]
    p["tw_amp"] = [0.0, 0.0, dT, 0.0]
    p["tw_k"] = [0.0, 0.0, 2.0 * math.pi / nx, 0.0]
    i, j = grid(nx, ny)
    y_if = ny / 2.0 - 0.5
    phi = tanh_profile(-(j - y_if), W)
    f = dict(phi=phi, ux=np.zeros_like(phi), uy=np.zeros_like(phi), T=np.full_like(phi, T0))
    return p, f


def heated_channel_table1(lambda_ratio: float = 1.0, W: float = 3.0) -> tuple[dict, dict]:
    """The heated channel at the size of the paper's Table 1 (Sec. 4.1):
    160 x 80 lattice, H = h = 40, lower wall T_h + T_0 cos(2 pi x / 160) with
    T_h = 20, T_0 = 4, upper wall T_c = 10, T_ref = 10, sigma_T = -5e-4,
    sigma_ref = 2.5e-2, rho = c_p = 1, mu = 0.2 in both fluids, lambda_h = 0.2,
    lambda_l = 0.2 lambda_ratio; light fluid on top.  Starts from the flat
    interface, u = 0 and the conduction profile between the wall means."""
    nx, ny = 160, 80
    Th, Tc, T0 = 20.0, 10.0, 4.0
    p, f = heated_channel(lambda_ratio, nx=nx, ny=ny, W=W, T0=Tc, dT=T0)
    p["tw_mean"] = [0.0, 0.0, Th, Tc]
    p["T_ref"] = 10.0
    j = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    f["T"] = Th + (Tc - Th) * (j + 0.5) / ny
    p["meta"] = dict(Th=Th, Tc=Tc, T0=T0, H=40.0, h=40.0, L=float(nx), lambda_r=lambda_ratio)
    return p, f


# ---------------------------------------------------------------------------
# Thermocapillary migration of a deformable droplet (Sec. 4.2)
# ---------------------------------------------------------------------------

def droplet(Ma: float = 0.1, ratio: float = 1.0, nx: int = 256, ny: int = 1024, R: float = 32.0,
            cy: float | None = None, Re: float = 0.5, mu_h: float = 0.05, lambda_h: float = 0.5,
            gradT: float | None = None, Ca_target: float | None = None,
            laplace_p: bool = False) -> tuple[dict, dict]:
    """Light droplet of radius R in a heavy fluid, periodic in x, walls at
    j = -1/2 and ny - 1/2 held at T = 0 and T = gradT * ny, linear initial T.
    With laplace_p the fields also carry p = (sigma_ref / R) (1 - phi) / 2, the
    Young-Laplace jump across the interface, so that a start from them does not
    emit the pressure wave of a start at p = 0.
    ratio scales the light phase's rho, mu, lambda and rho c_p.
    Ma = (rho c_p)_h R U / lambda_h, Re = R U / nu_h, U = -sigma_T gradT R / mu_h
    (characteristic scales of Sec. 4.2)."""
    if gradT is None:
        gradT = 8.0 / ny
    if cy is None:
        cy = ny / 4.0
    cx = nx / 2.0
    U = Re * mu_h / R                  # rho_h = 1
    sigma_T = -U * mu_h / (gradT * R)
    T_ref = gradT * (cy + 0.5)
    rhocp_h = Ma * lambda_h / (R * U)
    if Ca_target is None:
        sigma_ref = 2.0e-3 if (nx, ny, R) == (256, 1024, 32.0) else max(U * mu_h / 0.02,
                                                                        2.0 * abs(sigma_T) * gradT * 0.75 * ny)
    else:
        sigma_ref = U * mu_h / Ca_target
    p = base_params(nx, ny)
    p.update(bc=[PERIODIC, PERIODIC, WALL_T, WALL_T], W=3.0,
             rho_h=1.0, rho_l=ratio, mu_h=mu_h, mu_l=ratio * mu_h,
             lambda_h=lambda_h, lambda_l=ratio * lambda_h, rhocp_h=rhocp_h, rhocp_l=ratio * rhocp_h,
             sigma_ref=sigma_ref, sigma_T=sigma_T, sigma_TT=0.0, T_ref=T_ref)
    p["tw_mean"] = [0.0, 0.0, 0.0, gradT * ny]
    i, j = grid(nx, ny)
    r = np.sqrt((i - cx) ** 2 + (j - cy) ** 2)
    phi = tanh_profile(r - R, 3.0)
    T = gradT * (j + 0.5)
    f = dict(phi=phi, ux=np.zeros_like(phi), uy=np.zeros_like(phi), T=T)
    if laplace_p:
        f["p"] = (sigma_ref / R) * 0.5 * (1.0 - phi)
    meta = dict(U=U, R=R, gradT=gradT, mu_r=ratio, lambda_r=ratio, Ma=Ma, Re=Re,
                Ca=U * mu_h / sigma_ref, cx=cx, cy=cy)
    p["meta"] = meta
    return p, f


# ---------------------------------------------------------------------------
# Two recalcitrant bubbles with a parabolic sigma(T) (Sec. 4.3)
# ---------------------------------------------------------------------------

def droplet_table2(rho_ratio: float, nx: int = 160, ny: int = 320, R: float = 20.0) -> tuple[dict, dict]:
    """The density-ratio test of Sec. 4.2 (Table 2): light drop of radius 20
    at the centre of a 160 x 320 lattice, periodic in x, walls in y with the
    linear temperature of |grad T| = 0.1 from T_c = 16 at the bottom,
    rho_h = 1, rho_l = rho_h / rho_ratio, kinematic viscosity 0.8 in both
    fluids, (rho c_p)_h = 5, (rho c_p)_l = 1, lambda_h = 0.2, lambda_l = 0.1,
    sigma_ref = 2.5e-4, sigma_T = -1e-5 (the reading that reproduces every
    U_YGB of Table 2)."""
    gradT, Tc = 0.1, 16.0
    cx, cy = nx / 2.0, ny / 2.0
    nu = 0.8
    p = base_params(nx, ny)
    p.update(bc=[PERIODIC, PERIODIC, WALL_T, WALL_T], W=3.0,
             rho_h=1.0, rho_l=1.0 / rho_ratio, mu_h=nu, mu_l=nu / rho_ratio,
             lambda_h=0.2, lambda_l=0.1, rhocp_h=5.0, rhocp_l=1.0,
             sigma_ref=2.5e-4, sigma_T=-1e-5, sigma_TT=0.0, T_ref=Tc + gradT * (cy + 0.5))
    p["tw_mean"] = [0.0, 0.0, Tc, Tc + gradT * ny]
    i, j = grid(nx, ny)
    phi = tanh_profile(np.sqrt((i - cx) ** 2 + (j - cy) ** 2) - R, 3.0)
    f = dict(phi=phi, ux=np.zeros_like(phi), uy=np.zeros_like(phi), T=Tc + gradT * (j + 0.5))
    U = 1e-5 * gradT * R / nu
    p["meta"] = dict(U=U, R=R, gradT=gradT, rho_r=rho_ratio, mu_r=1.0 / rho_ratio, lambda_r=0.5, cx=cx, cy=cy)
    return p, f


def droplet_finite_ma(Ma: float, nx: int = 160, ny: int = 320, R: float = 20.0) -> tuple[dict, dict]:
    """The finite-Marangoni runs of Sec. 4.2 at Re = 1: the geometry of
    ``droplet_table2`` (drop of radius 20 at the centre, |grad T| = 0.1 from
    T_c = 16 at the bottom wall), equal densities 1, mu = 0.1 and lambda = 0.1
    in both fluids, sigma_ref = 5e-3, sigma_T = -2.5e-4, and Ma set through the
    heat capacitance of both fluids: U = -sigma_T |grad T| R / mu = 5e-3,
    Re = U R / nu = 1, Ma = rho c_p U R / lambda = rho c_p, Ca = 0.1.  The unit
    normal and grad T come from the stencils (grad_mode 1): with the normal
    from the moments, a mode seeded by rounding in the bulk grows at Ma >= 10
    and breaks the drop up after 12-35 R/U, at a time that depends on the
    rounding."""
    gradT, Tc = 0.1, 16.0
    cx, cy = nx / 2.0, ny / 2.0
    mu, lam, sigma_T = 0.1, 0.1, -2.5e-4
    U = -sigma_T * gradT * R / mu
    p = base_params(nx, ny)
    p.update(bc=[PERIODIC, PERIODIC, WALL_T, WALL_T], W=3.0, grad_mode=1,
             rho_h=1.0, rho_l=1.0, mu_h=mu, mu_l=mu, lambda_h=lam, lambda_l=lam,
             rhocp_h=Ma * lam / (U * R), rhocp_l=Ma * lam / (U * R),
             sigma_ref=5e-3, sigma_T=sigma_T, sigma_TT=0.0, T_ref=Tc + gradT * (cy + 0.5))
    p["tw_mean"] = [0.0, 0.0, Tc, Tc + gradT * ny]
    i, j = grid(nx, ny)
    phi = tanh_profile(np.sqrt((i - cx) ** 2 + (j - cy) ** 2) - R, 3.0)
    f = dict(phi=phi, ux=np.zeros_like(phi), uy=np.zeros_like(phi), T=Tc + gradT * (j + 0.5))
    p["meta"] = dict(U=U, R=R, gradT=gradT, Ma=Ma, Re=U * R / mu, Ca=U * mu / 5e-3, cx=cx, cy=cy)
    return p, f


def bubble_positions(nx: int, ny: int, radii=(24.0, 32.0), seed: int = 3):
    rng = np.random.default_rng(seed)
    while True:
        c = []
        for R in radii:
            x = rng.uniform(R + 16, nx - R - 16)
            y = rng.uniform(ny / 2.0, ny - R - 64)
            c.append((x, y))
        d = math.hypot(c[0][0] - c[1][0], c[0][1] - c[1][1])
        if d >= radii[0] + radii[1] + 12:
            return c


def two_bubbles(sigma_TT: float = 0.2, nx: int = 512, ny: int = 2048, radii=(24.0, 32.0),
                seed: int = 3) -> tuple[dict, dict]:
    """Flow along +y: inlet at j = -1/2, outlet at j = ny - 1/2, Dirichlet side
    walls with T_w(s) = 0.2 (s + 1/2) / ny bracketing T_ref = 0.1; density and
    viscosity ratio 10; sigma = sigma_ref + sigma_TT (T - T_ref)^2 / 2 (Eq. 63)."""
    p = base_params(nx, ny)
    Tslope = 0.2 / ny
    p.update(bc=[WALL_T, WALL_T, INLET, OUTLET], W=3.0,
             rho_h=1.0, rho_l=0.1, mu_h=0.04, mu_l=0.004,
             rhocp_h=20.0, rhocp_l=2.0, lambda_h=7.0, lambda_l=0.7,
             sigma_ref=2.5e-3, sigma_T=0.0, sigma_TT=sigma_TT, T_ref=0.1,
             u_in_mean=2.5e-4, phi_in=1.0, T_in=0.0)
    p["tw_mean"] = [0.5 * Tslope, 0.5 * Tslope, 0.0, 0.0]
    p["tw_slope"] = [Tslope, Tslope, 0.0, 0.0]
    cents = bubble_positions(nx, ny, radii, seed)
    p["bubbles_x"] = [c[0] for c in cents]
    p["bubbles_y"] = [c[1] for c in cents]
    i, j = grid(nx, ny)
    phi = np.ones((ny, nx))
    for (x0, y0), R in zip(cents, radii):
        phi = np.minimum(phi, tanh_profile(np.sqrt((i - x0) ** 2 + (j - y0) ** 2) - R, 3.0))
    xs = i + 0.5
    uy = 6.0 * p["u_in_mean"] * xs * (nx - xs) / nx ** 2
    T = Tslope * (j + 0.5)
    f = dict(phi=phi, ux=np.zeros_like(phi), uy=uy, T=T)
    return p, f


# ---------------------------------------------------------------------------
# Batched parameter sweep of droplet migrations of uneven lattice size
# ---------------------------------------------------------------------------

def sweep(n: int = 64, seed: int = 4, nx_range=(128, 256), laplace_p: bool = False) -> list[tuple[dict, dict]]:
    """n droplet-migration instances: NX uniform in nx_range, NY = 4 NX, drop at
    (NX/2, NY/4) with R uniform in [16, 40], Ma uniform in [0.1, 50], lambda_r
    uniform in [0.5, 2], rho = 1, mu = 0.05, lambda_h = 0.5 in both phases,
    rho c_p = 20 Ma in both phases.  laplace_p: start with the Young-Laplace
    pressure (see sweep_instance)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        ny = 4 * nx
        R = float(rng.uniform(16.0, 40.0))
        Ma = float(rng.uniform(0.1, 50.0))
        lr = float(rng.uniform(0.5, 2.0))
        out.append(sweep_instance(nx, ny, R, Ma, lr, laplace_p=laplace_p))
    return out


def sweep_instance(nx: int, ny: int, R: float, Ma: float, lambda_r: float,
                   laplace_p: bool = False) -> tuple[dict, dict]:
    mu, lam_h = 0.05, 0.5
    gradT = 8.0 / ny
    U = 0.5 * mu / R
    cx, cy = nx / 2.0, ny / 4.0
    sigma_T = -U * mu / (R * gradT)
    sigma_ref = max(U * mu / 0.02, 2.0 * abs(sigma_T) * gradT * 0.75 * ny)
    rhocp = Ma * lam_h / (R * U)
    p = base_params(nx, ny)
    p.update(bc=[PERIODIC, PERIODIC, WALL_T, WALL_T], W=3.0,
             rho_h=1.0, rho_l=1.0, mu_h=mu, mu_l=mu, lambda_h=lam_h, lambda_l=lam_h * lambda_r,
             rhocp_h=rhocp, rhocp_l=rhocp, sigma_ref=sigma_ref, sigma_T=sigma_T, sigma_TT=0.0,
             T_ref=gradT * (cy + 0.5))
    p["tw_mean"] = [0.0, 0.0, 0.0, gradT * ny]
    i, j = grid(nx, ny)
    phi = tanh_profile(np.sqrt((i - cx) ** 2 + (j - cy) ** 2) - R, 3.0)
    f = dict(phi=phi, ux=np.zeros_like(phi), uy=np.zeros_like(phi), T=gradT * (j + 0.5))
    if laplace_p:
        f["p"] = (sigma_ref / R) * 0.5 * (1.0 - phi)
    p["meta"] = dict(U=U, R=R, Ma=Ma, lambda_r=lambda_r, gradT=gradT, cx=cx, cy=cy)
    return p, f


# ---------------------------------------------------------------------------
# Small cases for parity and unit tests
# ---------------------------------------------------------------------------

def tiny(nx: int, ny: int, bc=(PERIODIC, PERIODIC, WALL_T, WALL_T), seed: int = 0,
         rho_ratio: float = 0.5, sigma_TT: float = 0.0) -> tuple[dict, dict]:
    """A small lattice with one circular light droplet, property contrasts in
    every quantity, a nonzero velocity field and a wall temperature with both
    cosine and linear parts on every non-periodic side."""
    rng = np.random.default_rng(seed)
    p = base_params(nx, ny)
    p.update(bc=list(bc), W=2.0 if min(nx, ny) < 16 else 3.0,
             rho_h=1.0, rho_l=rho_ratio, mu_h=0.08, mu_l=0.05, lambda_h=0.3, lambda_l=0.15,
             rhocp_h=3.0, rhocp_l=1.5, sigma_ref=5e-3, sigma_T=-2e-4, sigma_TT=sigma_TT, T_ref=1.0,
             mobility=0.08, Gx=1e-6, Gy=-2e-6, u_in_mean=1e-3, phi_in=1.0, T_in=0.8)
    for s in range(4):
        L = ny if s < 2 else nx
        p["tw_mean"][s] = 1.0 + 0.1 * s
        p["tw_amp"][s] = 0.2
        p["tw_k"][s] = 2.0 * math.pi / L
        p["tw_slope"][s] = 0.01
    i, j = grid(nx, ny)
    cx = nx / 2.0 + rng.uniform(-1, 1)
    cy = ny / 2.0 + rng.uniform(-1, 1)
    R = 0.3 * min(nx, ny)
    phi = tanh_profile(np.sqrt((i - cx) ** 2 + (j - cy) ** 2) - R, p["W"])
    ux = 1e-3 * np.sin(2 * math.pi * j / ny + rng.uniform(0, 6)) * (1 + 0.1 * rng.standard_normal((ny, nx)))
    uy = 1e-3 * np.cos(2 * math.pi * i / nx + rng.uniform(0, 6)) * (1 + 0.1 * rng.standard_normal((ny, nx)))
    T = 1.0 + 0.2 * np.sin(2 * math.pi * i / nx) * np.cos(math.pi * j / ny) + 0.05 * rng.standard_normal((ny, nx))
    p["bubbles_x"] = [cx]
    p["bubbles_y"] = [cy]
    return p, dict(phi=phi, ux=ux, uy=uy, T=T)


def perturbation(nx: int, ny: int, seed: int = 1, scale: float = 1e-3) -> dict:
    """Random population offsets for single-step parity tests: arrays f, g, h of
    shape (9, ny, nx) and jprev of shape (2, ny, nx), to be added to a state."""
    rng = np.random.default_rng(seed)
    return dict(f=scale * rng.standard_normal((9, ny, nx)),
                g=scale * rng.standard_normal((9, ny, nx)),
                h=scale * rng.standard_normal((9, ny, nx)),
                jprev=scale * rng.standard_normal((2, ny, nx)))


ALL_BCS = [
    (PERIODIC, PERIODIC, PERIODIC, PERIODIC),
    (PERIODIC, PERIODIC, WALL_T, WALL_T),
    (PERIODIC, PERIODIC, WALL_ADIABATIC, WALL_T),
    (WALL_T, WALL_ADIABATIC, PERIODIC, PERIODIC),
    (WALL_T, WALL_T, INLET, OUTLET),
    (WALL_ADIABATIC, WALL_T, WALL_T, WALL_ADIABATIC),
]

"""Closed-form results the paper states, used to pin the oracle.

TEST INFRASTRUCTURE (see the package docstring).

* ``channel_solution``: steady temperature and velocity of two superimposed
  planar fluids in a heated microchannel (Pendse & Esmaeeli closed form quoted
  in Sec. 4.1).
* ``u_ygb``: terminal thermocapillary migration velocity of a drop at vanishing
  Re and Ma (Eq. 60), with U = -sigma_T |grad T| R / mu_h (Sec. 4.2).
* ``u_2d``: the same balance for a circular (2-D) drop, derived from the 2-D
  Stokes streamfunction (not in the paper; it is the geometry the paper's 2-D
  runs actually have).
* ``groups``: dimensionless numbers of Eq. 46.
* ``rel_l2``: the relative error E_delta of the Table 1 caption.
"""
from __future__ import annotations

import math

import numpy as np


def channel_solution(x, y, *, L, H, h, Tc, Th, T0, lambda_r, mu_r, sigma_T, mu_h):
    """Steady fields of Sec. 4.1.  y is measured from the interface: the light
    layer occupies 0 <= y <= H, the heavy layer -h <= y <= 0.  The lower wall is
    at Th + T0 cos(2 pi x / L), the upper wall at Tc.  lambda_r = lambda_l /
    lambda_h, mu_r = mu_l / mu_h.  Returns (T, ux, uy) arrays."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = 2.0 * math.pi / L
    Ht, ht = w * H, w * h
    fH = 1.0 / (lambda_r * math.sinh(ht) * math.cosh(Ht) + math.sinh(Ht) * math.cosh(ht))
    DH = math.sinh(Ht) ** 2 - Ht ** 2
    Dh = math.sinh(ht) ** 2 - ht ** 2
    C1H, C2H, C3H = math.sinh(Ht) ** 2 / DH, -H * Ht / DH, (2 * Ht - math.sinh(2 * Ht)) / (2 * DH)
    C1h, C2h, C3h = math.sinh(ht) ** 2 / Dh, -h * ht / Dh, (math.sinh(2 * ht) - 2 * ht) / (2 * Dh)
    g = math.sinh(Ht) * fH
    hfn = DH * Dh / (mu_r * Dh * (math.sinh(2 * Ht) - 2 * Ht) + DH * (math.sinh(2 * ht) - 2 * ht))
    Umax = -(T0 * sigma_T / mu_h) * g * hfn
    den = H + lambda_r * h
    TL = ((Tc - Th) * y + lambda_r * Tc * h + Th * H) / den + T0 * fH * np.sinh(Ht - w * y) * np.cos(w * x)
    TH = ((lambda_r * (Tc - Th) * y + lambda_r * Tc * h + Th * H) / den
          + T0 * fH * (math.sinh(Ht) * np.cosh(w * y) - lambda_r * np.sinh(w * y) * math.cosh(Ht)) * np.cos(w * x))

    def ux_of(C1, C2, C3):
        return Umax * ((C1 + w * (C2 + C3 * y)) * np.cosh(w * y) + (C3 + w * C1 * y) * np.sinh(w * y)) * np.sin(w * x)

    def uy_of(C1, C2, C3):
        return -w * Umax * (C1 * y * np.cosh(w * y) + (C2 + C3 * y) * np.sinh(w * y)) * np.cos(w * x)

    upper = y >= 0
    T = np.where(upper, TL, TH)
    ux = np.where(upper, ux_of(C1H, C2H, C3H), ux_of(C1h, C2h, C3h))
    uy = np.where(upper, uy_of(C1H, C2H, C3H), uy_of(C1h, C2h, C3h))
    return T, ux, uy, dict(Umax=Umax, f=fH, g=g, hfn=hfn)


def u_char(sigma_T: float, gradT: float, R: float, mu_h: float) -> float:
    """Characteristic thermocapillary velocity U = -sigma_T |grad T| R / mu_h."""
    return -sigma_T * abs(gradT) * R / mu_h


def u_ygb(U: float, mu_r: float, lambda_r: float) -> float:
    """Eq. 60: U_YGB = 2 U / ((2 + 3 mu_r)(2 + lambda_r))."""
    return 2.0 * U / ((2.0 + 3.0 * mu_r) * (2.0 + lambda_r))


def u_2d(U: float, mu_r: float, lambda_r: float) -> float:
    """Circular drop in 2-D Stokes flow: U / (2 (1 + mu_r)(1 + lambda_r))."""
    return U / (2.0 * (1.0 + mu_r) * (1.0 + lambda_r))


def groups(*, L, U, nu_h, rho_h, cp_h, lambda_h, mu_h, sigma_ref) -> dict:
    """Eq. 46: Re = L U / nu_h, Ma = rho_h c_p,h L U / lambda_h, Ca = U mu_h / sigma_ref."""
    return dict(Re=L * U / nu_h, Ma=rho_h * cp_h * L * U / lambda_h, Ca=U * mu_h / sigma_ref)


def rel_l2(num, ana) -> float:
    """E_delta = sqrt(sum |xi_n - xi_a|^2 / sum |xi_a|^2) (Table 1 caption)."""
    num = np.asarray(num, dtype=np.float64)
    ana = np.asarray(ana, dtype=np.float64)
    return float(np.sqrt(np.sum((num - ana) ** 2) / np.sum(ana ** 2)))

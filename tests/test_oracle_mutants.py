"""The oracle's pins catch plausible mistakes: each case plants one mistake in
a copy of the oracle's C source (or of the reference Adam step), builds it on
the CPU and checks that the pin written for that part fails on it, while the
unmodified oracle passes the same pin (the pins' own tests).

Planted mistakes: a dropped factor 1/2 in the parabolic term of Eq. 63, T_ref
dropped from sigma'(T), a sign error in sigma'(T), the farthest centroid in
place of the nearest one in the region split of Sec. 4.3, ties sent to the
higher region, a region's x centroid summed over y; for the channel of Sec.
4.3, the inflow profile scaled by 4 instead of 6, the inflow velocity with the
wrong sign, an outlet that copies the node's own post-collision population
(a zero-gradient reading) and an outlet that bounces back like a wall; and,
for Adam, a missing bias correction, swapped decay rates and a bias
correction one step late.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import conv_ref as cr
from tests import test_oracle_conv as tconv
from tests import test_oracle_pins as tpins
from tests import test_oracle_sigma_regions as tsr

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "lbm_oracle.c")).read()

MUTANTS = {
    "sigma_half_dropped": ("0.5 * P->sigma_TT * d * d", "P->sigma_TT * d * d",
                           [tsr.test_parabolic_sigma_laplace_jump]),
    "dsigma_no_Tref": ("P->sigma_TT * (T - P->T_ref)", "P->sigma_TT * T",
                       [lambda: tsr.test_parabolic_sigma_tangential_force(0.0, 2e-3)]),
    "dsigma_sign": ("return P->sigma_T + P->sigma_TT", "return P->sigma_T - P->sigma_TT",
                    [lambda: tsr.test_parabolic_sigma_tangential_force(-5e-4, 2e-3)]),
    "farthest_centroid": ("if (b == 0 || d2 < bd)", "if (b == 0 || d2 > bd)",
                          [tsr.test_regions_follow_the_nearest_previous_centroid]),
    "ties_to_higher": ("if (b == 0 || d2 < bd)", "if (b == 0 || d2 <= bd)",
                       [tsr.test_regions_tie_and_empty_region, tsr.test_regions_split_equidistant_column]),
    "region_x_from_y": ("bxs[best] += phi * i;", "bxs[best] += phi * j;",
                        [lambda: tsr.test_regions_two_static_drops((0, 1))]),
    "inflow_profile_scale": ("double un = 6.0 * P->u_in", "double un = 4.0 * P->u_in",
                             [tpins.check_channel_flow]),
    "inflow_sign": ("gb = gs[k] - 2.0 * WI[k] * rho", "gb = gs[k] + 2.0 * WI[k] * rho",
                    [tpins.check_channel_flow]),
    "outlet_copy": ("gb = -gs[k] + 2.0 * WI[k] * rho * (cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));",
                    "gb = gs[kb] + 0.0 * rho * cu * uu;", [tpins.check_channel_flow]),
    "outlet_closed": ("gb = -gs[k] + 2.0 * WI[k] * rho * (cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));",
                      "gb = gs[k] + 0.0 * rho * cu * uu;", [tpins.check_channel_flow]),
}


@pytest.fixture(scope="module")
def built(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_mutants")
    out = {}
    for name, (old, new, _) in MUTANTS.items():
        assert SRC.count(old) == 1, f"mutation site of {name} not unique"
        out[name] = oracle.build_variant(SRC.replace(old, new), str(d / f"lib_{name}.so"))
    return out


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pin_catches_planted_mistake(name, built):
    _, _, pins = MUTANTS[name]
    with oracle.use_library(built[name]):
        for pin in pins:
            with pytest.raises(AssertionError):
                pin()


def _adam_no_bias(p, g, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    return p - lr * m1 / (np.sqrt(m2) + eps), m1, m2


def _adam_swapped(p, g, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    return cr.adam(p, g, m1, m2, t, lr=lr, b1=b2, b2=b1, eps=eps)


def _adam_late(p, g, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    tt = max(t - 1, 1)
    return p - lr * (m1 / (1 - b1 ** tt)) / (np.sqrt(m2 / (1 - b2 ** tt)) + eps), m1, m2


@pytest.mark.parametrize("mutant", [_adam_no_bias, _adam_swapped, _adam_late], ids=["no_bias", "swapped", "late"])
def test_adam_pins_catch_planted_mistake(mutant):
    failures = 0
    for pin in (tconv.check_adam_constant_gradient, tconv.check_adam_impulse_response):
        try:
            pin(mutant)
        except AssertionError:
            failures += 1
    assert failures >= 1

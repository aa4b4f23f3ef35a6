"""The paper's water models (Sec. IV, Tables I-III) as workloads: hierarchy
sizes and the reading of the tables' normalisations (CPU, oracle only).

The caption relations x~ = f x between the tabulated and the model values
are applied as x = f x~; the checks below are what fixes that direction: the
kept levels must lie inside the well of each mode's cubic potential and the
modes must be weakly anharmonic, which the literal direction violates for the
bend.
"""

import math

import numpy as np

import workloads as w
from oracle import hierarchy as oy
from oracle import model as om


def test_water_hierarchy_sizes():
    # K = 4 Pade terms per mode: M = 2 x 5 = 10 (two modes), 3 x 5 = 15
    # (three); the triangular set |n| <= L has C(M + L, L) members (the
    # enumeration is checked against the binomial at a size it can list)
    assert len(oy.enumerate_ados(10, 2)) == math.comb(12, 2) == 66
    assert math.comb(10 + 4, 4) == 1001
    assert math.comb(15 + 4, 4) == 3876
    assert math.comb(15 + 5, 5) == 15504
    for f, n_modes in ((w.water_two_mode, 2), (w.water_three_mode, 3)):
        for levels in (3, 4):
            p = f(n_levels=levels, depth=1)
            o = om.build(p)
            assert o.d == levels ** n_modes
            assert len(o.nu) == 5 * n_modes
            assert len(o.hier) == 1 + 5 * n_modes


def test_water_time_step_and_temperature():
    p = w.water_two_mode()
    assert abs(p["dt"] * w.FS_PER_TIME_UNIT_WATER - 0.25) < 1e-12
    # 300 K: k_B T = 208.51 cm^-1
    assert abs(w.WATER_OMEGA0_CM / p["beta"] - 208.5104) < 1e-3
    assert [m["omega"] * w.WATER_OMEGA0_CM for m in w.water_three_mode()["modes"]] == \
        [3570.0, 3470.0, 1710.0]


def _barrier(omega, g3):
    # omega q^2/2 + g3 q^3/6 has its local maximum at q = -2 omega/g3, height
    # (2/3) omega^3 / g3^2 above the minimum
    return 2.0 * omega ** 3 / (3.0 * g3 * g3)


def test_water_modes_bound_and_weakly_anharmonic():
    for f in (w.water_two_mode, w.water_three_mode):
        p = f()
        for md in p["modes"]:
            om_, g3 = md["omega"], md["g3"]
            r = om_ / 1.0   # omega_s / omega0
            # the kept levels lie inside the well (harmonic estimate of the
            # highest kept level above the minimum)
            assert _barrier(om_, g3) > (md["n_keep"] - 0.5) * om_
            # isolated mode (no bath, so no counter term; a 20-level basis,
            # which converges the kept levels of a cubic well to 1e-6):
            # fundamental within 5% below the harmonic frequency, and equal
            # to the second-order perturbative value omega - 5 g3^2/(24 omega)
            # up to the next order (5e-3)
            iso = dict(md, zeta=0.0, n_basis=20, n_keep=md["n_keep"])
            E = om.single_mode(iso).E
            gap = E[1] - E[0]
            assert 0.95 * om_ < gap < om_
            assert abs(gap - (om_ - 5 * g3 * g3 / (24 * om_))) < 5e-3
            # the literal direction of the caption (g3 = g~ / r^3 = g3 / r^6)
            # leaves no bound level in the bend
            if r < 0.5:
                assert _barrier(om_, g3 / r ** 6) < 0.5 * om_

"""Pins of the oracle's macroscopic theory against numbers the paper prints
(tests/golden/paper_printed.json) and against closed forms."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import analytics as A
from paper_2003_07968_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed.json")))


def test_paper_eos_critical_point_is_unity():
    # The paper uses T directly as the reduced temperature T_r with the Sec. IV.A
    # constants (and prints Maxwell values at "T_r = 0.8" computed at T = 0.8),
    # which requires rho_c = T_c = 1 for that set.
    rho_c, T_c, p_c = A.critical_point(A.PAPER_EOS)
    assert abs(rho_c - 1.0) < 1e-6
    assert abs(T_c - 1.0) < 1e-6
    # both derivatives vanish there
    assert abs(A.PAPER_EOS.dP(rho_c, T_c)) < 1e-10
    assert abs(A.PAPER_EOS.d2P(rho_c, T_c)) < 1e-8


def test_eos_derivatives_match_finite_differences():
    eos = A.UNIT_EOS
    for rho in (0.01, 0.1, 0.3, 0.45):
        h = 1e-6
        fd1 = (eos.P(rho + h, 0.07) - eos.P(rho - h, 0.07)) / (2 * h)
        fd2 = (eos.dP(rho + h, 0.07) - eos.dP(rho - h, 0.07)) / (2 * h)
        assert abs(eos.dP(rho, 0.07) - fd1) < 1e-7 * max(1, abs(fd1))
        assert abs(eos.d2P(rho, 0.07) - fd2) < 1e-6 * max(1, abs(fd2))


def test_unit_eos_critical_point_matches_scaling():
    # With e = b rho, Eq. CSEOS reads k [(c/b) e T Z(e) - (a/b^2) e^2], so
    # rho_c = rho_c(unit)/b and T_c = T_c(unit) a/(b c).  With the paper's set
    # this maps the unit set's critical point onto (1, 1).
    rho_c1, T_c1, _ = A.critical_point(A.UNIT_EOS)
    assert abs(rho_c1 / A.PAPER_EOS.b - 1.0) < 1e-6
    assert abs(T_c1 * A.PAPER_EOS.a / (A.PAPER_EOS.b * A.PAPER_EOS.c) - 1.0) < 1e-6
    assert abs(T_c1 - W.UNIT_CS_TC) < 1e-12
    assert abs(rho_c1 - W.UNIT_CS_RHOC) < 1e-12


def test_maxwell_printed_values():
    g = GOLD["maxwell_Tr0.8"]
    rg, rl, p0 = A.maxwell(A.PAPER_EOS, g["T_r"])
    assert round(rg, 4) == g["rho_g"]
    assert round(rl, 4) == g["rho_l"]
    # equal pressures and equal areas
    assert abs(A.PAPER_EOS.P(rg, 0.8) - p0) < 1e-14
    assert abs(A.PAPER_EOS.P(rl, 0.8) - p0) < 1e-14


def test_maxwell_equal_area_closed_form():
    # Independent route: the CS free energy gives int P/rho^2 drho in closed
    # form, k [c T (ln(e) + (4e - 3e^2)/(1 - e)^2) - a rho], e = b rho.
    eos = A.PAPER_EOS
    T = 0.7
    rg, rl, p0 = A.maxwell(eos, T)

    def prim(rho):
        e = eos.b * rho
        return eos.k * (eos.c * T * (math.log(e) + (4 * e - 3 * e * e) / (1 - e) ** 2)
                        - eos.a * rho)

    area = p0 * (1 / rg - 1 / rl) - (prim(rl) - prim(rg))
    assert abs(area) < 1e-10 * p0 / rg


def test_mechanical_coexistence_printed_values():
    g = GOLD["mechanical_Tr0.8_eps1.73"]
    rg, rl, p0 = A.mechanical_coexistence(A.PAPER_EOS, g["T_r"], g["epsilon"])
    # printed with "approximately"; agree to one unit in the last printed digit
    assert abs(rg - g["rho_g"]) <= 1e-4
    assert abs(rl - g["rho_l"]) <= 1e-4


def test_mechanical_coexistence_independent_of_G_scale():
    # psi scales as |G|^(-1/2), so psi_dot / psi^(1+eps) scales by a constant.
    a = A.mechanical_coexistence(A.PAPER_EOS, 0.8, 1.73, G=-1.0)
    b = A.mechanical_coexistence(A.PAPER_EOS, 0.8, 1.73, G=-5.0)
    assert np.allclose(a[:2], b[:2], rtol=1e-9)


def test_eps_zero_is_shan_chen_far_from_maxwell():
    # eps = 0 is the Shan-Chen force; its gas branch is far below Maxwell's,
    # which is the deficiency the paper's eps corrects (Sec. IV.A).
    rg0, rl0, _ = A.mechanical_coexistence(A.PAPER_EOS, 0.8, 0.0)
    rgm, rlm, _ = A.maxwell(A.PAPER_EOS, 0.8)
    assert rg0 < 0.5 * rgm
    # eps = 1.73 brings the planar densities to within 6 % of Maxwell
    rg, rl, _ = A.mechanical_coexistence(A.PAPER_EOS, 0.8, 1.73)
    assert abs(rg / rgm - 1) < 0.06 and abs(rl / rlm - 1) < 0.002


def test_planar_surface_tension_printed_value():
    g = GOLD["planar_surface_tension"]
    quad = A.planar_surface_tension_quad(A.PAPER_EOS, g["T_r"], g["epsilon"], 1.0)
    # The paper prints three significant digits from its own FD + Newton run;
    # both routes here land within 1.5 % of it and within 0.5 % of each other.
    assert abs(quad / g["gamma_pi_per_sigma"] - 1) < 0.015
    for dx in g["dx"]:
        fd = A.planar_surface_tension_fd(A.PAPER_EOS, g["T_r"], g["epsilon"], 1.0, L=g["L"],
                                         dx=dx)
        assert abs(fd / g["gamma_pi_per_sigma"] - 1) < 0.015
        assert abs(fd / quad - 1) < 0.005


def test_planar_surface_tension_scales_with_sigma_table():
    g = GOLD["planar_surface_tension"]
    base = A.planar_surface_tension_quad(A.PAPER_EOS, g["T_r"], g["epsilon"], 1.0)
    for s, printed in zip(g["table_sigma"], g["table_gamma_pi"]):
        val = A.planar_surface_tension_quad(A.PAPER_EOS, g["T_r"], g["epsilon"], s)
        assert abs(val - s * base) < 1e-12
        assert abs(val / printed - 1) < 0.015


def test_planar_profile_satisfies_first_integral_at_ends():
    # y(psi_l) = psi'^2 at the liquid side vanishes exactly when Eq. PGLDR holds.
    x, rho, psi, p0 = A.planar_profile_fd(A.PAPER_EOS, 0.8, 1.73, dx=0.1)
    d = np.gradient(psi, x)
    assert abs(d[0]) < 0.01 * abs(d).max() and abs(d[-1]) < 0.01 * abs(d).max()
    assert np.all(np.diff(rho) > 0)


def test_lamb_period_printed_values():
    g = GOLD["lamb_period"]
    for case in g["cases"]:
        Ta = A.lamb_period(case["gamma"], case["rho_l"], g["R_max"], g["R_min"], g["n"])
        assert round(Ta) == case["T_a"]


def test_workload_coexistence_table_is_maxwell():
    for tr, (rg, rl) in W.UNIT_CS_MAXWELL.items():
        mg, ml, _ = A.maxwell(A.UNIT_EOS, tr * W.UNIT_CS_TC)
        assert abs(mg / rg - 1) < 1e-9 and abs(ml / rl - 1) < 1e-9


def test_psi_real_between_phases():
    # Eq. DED needs (P - cs^2 rho)/G >= 0 over the whole coexistence range.
    for tr in (0.6, 0.7, 0.8, 0.9):
        T = tr * W.UNIT_CS_TC
        rg, rl = W.unit_cs_coexistence(tr)
        rho = np.linspace(rg * 0.5, rl * 1.1, 200)
        assert np.all((A.UNIT_EOS.P(rho, T) - rho / 3) / -1.0 > 0)


class ConsistentEOS:
    """An equation of state for which the consistency condition of Eq. CTC
    holds exactly: P = cs^2 rho + G psi^2 with psi = (T/rho + 1)^(-1/eps0) and
    G = -1, so that psi_dot / psi^(1 + eps0) = T / (eps0 rho^2).  Eq. PGLDR at
    eps = eps0 is then Maxwell's rule (Eq. MLVDR) term by term, for both
    densities, and the fit of eps must return eps0 (a closed form written here
    without the oracle's EOS code)."""

    rho_max = 1e3

    def __init__(self, eps0):
        self.eps0 = eps0

    def P(self, rho, T):
        return rho / 3.0 - (T / rho + 1.0) ** (-2.0 / self.eps0)

    def dP(self, rho, T):
        return 1.0 / 3.0 - (2.0 / self.eps0) * (T / rho + 1.0) ** (-2.0 / self.eps0 - 1) * T / rho**2

    def spinodals(self, T):
        from scipy import optimize
        grid = np.geomspace(1e-6, 1e2, 20001)
        d = self.dP(grid, T)
        idx = np.where(np.sign(d[:-1]) != np.sign(d[1:]))[0]
        assert len(idx) == 2
        return tuple(optimize.brentq(lambda r: self.dP(r, T), grid[i], grid[i + 1], xtol=1e-15)
                     for i in idx)


@pytest.mark.parametrize("eps0,T", [(1.2, 1.0), (1.5, 1.5)])
def test_fit_epsilon_recovers_exactly_consistent_eos(eps0, T):
    eos = ConsistentEOS(eps0)
    rgm, rlm, p0m = A.maxwell(eos, T)
    assert 0.05 < rgm / rlm < 0.5          # a genuine two-phase state
    rg, rl, p0 = A.mechanical_coexistence(eos, T, eps0)
    assert abs(rg / rgm - 1) < 1e-10 and abs(rl / rlm - 1) < 1e-10
    assert abs(A.fit_epsilon(eos, T, lo=0.8, hi=2.4) - eps0) < 1e-8
    # one step off eps0 the two constructions part
    rg2, rl2, _ = A.mechanical_coexistence(eos, T, eps0 + 0.02)
    assert abs(rg2 / rgm - 1) > 1e-4


@pytest.mark.parametrize("eos_name,tr", [("paper", 0.6), ("paper", 0.8), ("paper", 0.9),
                                         ("unit", 0.7), ("unit", 0.8), ("unit", 0.9)])
def test_fit_epsilon_matches_both_maxwell_densities(eos_name, tr):
    # The fit matches the Maxwell liquid density (Eq. CTC imposed at one
    # temperature).  Both coexistence densities are roots of P = p0, so once
    # the liquid one matches, p0 and with it the gas density match too: a
    # wrong root or a wrong branch of the scan fails the 1e-8 bar on one of
    # them.
    eos, Tc = (A.PAPER_EOS, 1.0) if eos_name == "paper" else (A.UNIT_EOS, W.UNIT_CS_TC)
    T = tr * Tc
    eps = A.fit_epsilon(eos, T)
    rgm, rlm, _ = A.maxwell(eos, T)
    rg, rl, _ = A.mechanical_coexistence(eos, T, eps)
    assert abs(rl / rlm - 1) < 1e-8
    assert abs(rg / rgm - 1) < 1e-8


def test_fit_epsilon_side_fixed_by_printed_densities():
    # Sec. IV.B prints the planar densities at eps = 1.73 (0.1580 / 2.3530)
    # below the Maxwell ones (0.1665 / 2.3550) at T_r = 0.8.  Both planar
    # densities grow with eps, so the eps that reaches Maxwell lies above
    # 1.73: the analytic fit gives 1.90 on the paper's EOS (the paper chose
    # 1.73 by adjusting lattice runs, not Eq. PGLDR).
    pg = GOLD["mechanical_Tr0.8_eps1.73"]
    mw = GOLD["maxwell_Tr0.8"]
    assert pg["rho_l"] < mw["rho_l"] and pg["rho_g"] < mw["rho_g"]
    grid = [1.6, 1.7, 1.8, 1.9, 2.0]
    dens = [A.mechanical_coexistence(A.PAPER_EOS, 0.8, e)[:2] for e in grid]
    assert all(b[0] > a[0] and b[1] > a[1] for a, b in zip(dens, dens[1:]))
    eps = A.fit_epsilon(A.PAPER_EOS, 0.8)
    assert 1.73 < eps < 2.0
    assert abs(eps - 1.9028) < 1e-3


def test_quadrature_of_pgldr_matches_trapezoid():
    # The PGLDR integral at the solution is ~0 by construction; recompute it by
    # a dense trapezoid rule as an independent integrator.
    eos, T, eps = A.PAPER_EOS, 0.8, 1.73
    rg, rl, p0 = A.mechanical_coexistence(eos, T, eps)
    r = np.linspace(rg, rl, 400001)
    fn = (p0 - eos.P(r, T)) * A.dpsi_drho(eos, T, r) / A.psi_of_rho(eos, T, r) ** (1 + eps)
    scale = integrate.trapezoid(np.abs(fn), r)
    assert abs(integrate.trapezoid(fn, r)) < 1e-8 * scale

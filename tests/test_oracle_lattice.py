"""Pins of the lattice oracle's pointwise pieces and force stencils against
closed forms, the paper's Appendix A moments, the continuum expansions of
Secs. II.C and III.B-C, and separately written special cases."""
import math

import numpy as np
import pytest

from paper_2003_07968_amd import workloads as W

from .helpers import oracle_params

CS2 = 1.0 / 3.0

# D2Q9 velocities (Eq. VelocitySet), written out here for the moment checks.
C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
             dtype=float)

# The Gram-Schmidt MRT matrix of Appendix A (Eq. MatrixMRT).
M_MRT = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=float)


def test_equilibrium_hydrodynamic_moments(oracle):
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho = rng.uniform(0.01, 3.0)
        u = rng.uniform(-0.2, 0.2, size=2)
        feq = oracle.equilibrium(rho, *u)
        assert abs(feq.sum() - rho) < 1e-15 * rho * 10
        assert np.allclose(feq @ C, rho * u, atol=1e-15 * rho * 10, rtol=0)
        second = np.einsum("i,ia,ib->ab", feq, C, C)
        assert np.allclose(second, rho * CS2 * np.eye(2) + rho * np.outer(u, u),
                           atol=1e-15 * rho * 10, rtol=0)


def test_equilibrium_mrt_moments_appendix_a(oracle):
    # m_eq = M f_eq, Appendix A
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.01, 3.0)
        ux, uy = rng.uniform(-0.2, 0.2, size=2)
        m = M_MRT @ oracle.equilibrium(rho, ux, uy)
        u2 = ux * ux + uy * uy
        expect = [rho, -2 * rho + 3 * rho * u2, rho - 3 * rho * u2, rho * ux, -rho * ux,
                  rho * uy, -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy]
        assert np.allclose(m, expect, atol=1e-14 * max(1, rho), rtol=0)


def test_guo_source_moments_and_appendix_a(oracle):
    rng = np.random.default_rng(2)
    for _ in range(20):
        tau = rng.uniform(0.51, 2.0)
        ux, uy, Fx, Fy = rng.uniform(-0.1, 0.1, size=4)
        S = oracle.guo_source(tau, ux, uy, Fx, Fy)
        fac = 1 - 1 / (2 * tau)
        assert abs(S.sum()) < 1e-16
        assert np.allclose(S @ C, fac * np.array([Fx, Fy]), atol=1e-16, rtol=0)
        # Appendix A: S_bar = M S for the Guo term without the BGK factor
        Sbar = M_MRT @ (S / fac)
        uF = ux * Fx + uy * Fy
        expect = [0, 6 * uF, -6 * uF, Fx, -Fx, Fy, -Fy, 2 * (ux * Fx - uy * Fy),
                  ux * Fy + uy * Fx]
        assert np.allclose(Sbar, expect, atol=1e-16, rtol=0)


def _plane_wave(nx, ny, mx, my, phase, a0=1.0, a1=0.2):
    kx, ky = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    th = kx * x + ky * y + phase
    return kx, ky, th, a0 + a1 * np.cos(th)


@pytest.mark.parametrize("mx,my", [(1, 0), (0, 1), (2, 3), (5, 1)])
def test_psi_moments_fourier_closed_form(oracle, mx, my):
    # For psi = a0 + a1 cos(theta), theta = k.x + phase, each moment is a trig
    # polynomial in (kx, ky) obtained by summing the nine shifted cosines.
    nx, ny = 24, 20
    kx, ky, th, psi = _plane_wave(nx, ny, mx, my, 0.37)
    m = oracle.psi_moments(psi)
    a1 = 0.2
    cx, cy, sx, sy = math.cos(kx), math.cos(ky), math.sin(kx), math.sin(ky)
    M0 = 1.0 + a1 * np.cos(th) * (4 / 9 + 2 / 9 * (cx + cy) + cx * cy / 9)
    M1x = -a1 * np.sin(th) * sx * (2 + cy) / 9
    M1y = -a1 * np.sin(th) * sy * (2 + cx) / 9
    M2xx = a1 * np.cos(th) * (-4 / 27 + 4 / 27 * cx - 2 / 27 * cy + 2 / 27 * cx * cy)
    M2yy = a1 * np.cos(th) * (-4 / 27 + 4 / 27 * cy - 2 / 27 * cx + 2 / 27 * cx * cy)
    M2xy = -a1 * np.cos(th) * sx * sy / 9
    for name, ref in [("M0", M0), ("M1x", M1x), ("M1y", M1y), ("M2xx", M2xx), ("M2yy", M2yy),
                      ("M2xy", M2xy)]:
        assert np.allclose(m[name], ref, atol=2e-16 * 10, rtol=0), name


def test_psi_moments_taylor_forms(oracle):
    # Eqs. ZOMED, FOMED, SOMED: for a smooth field the moments approach
    # psi + cs^2/2 Lap psi, cs^2 grad psi + cs^4/2 grad Lap psi and
    # cs^4 grad grad psi; the neglected terms are two orders higher.
    errs = []
    for n in (32, 64, 128):
        kx = ky = 2 * np.pi / n
        y, x = np.mgrid[0:n, 0:n].astype(float)
        psi = 1.0 + 0.3 * np.sin(kx * x) * np.cos(ky * y)
        m = oracle.psi_moments(psi)
        s, c = np.sin(kx * x), np.cos(ky * y)
        lap = -0.3 * (kx**2 + ky**2) * s * c
        dx = 0.3 * kx * np.cos(kx * x) * c
        dxx = -0.3 * kx**2 * s * c
        dxy = -0.3 * kx * ky * np.cos(kx * x) * np.sin(ky * y)
        dx_lap = -(kx**2 + ky**2) * dx
        e0 = np.abs(m["M0"] - (psi + CS2 / 2 * lap)).max() / np.abs(lap).max()
        e1 = np.abs(m["M1x"] - (CS2 * dx + CS2**2 / 2 * dx_lap)).max() / np.abs(dx).max()
        e2 = np.abs(m["M2xx"] - CS2**2 * dxx).max() / np.abs(dxx).max()
        e3 = np.abs(m["M2xy"] - CS2**2 * dxy).max() / np.abs(dxy).max()
        errs.append((e0, e1, e2, e3))
    errs = np.array(errs)
    # relative error falls by ~4x (second order) per halving of k
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.5), ratios


def _random_psi(nx, ny, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.2, 1.0, size=(ny, nx))


@pytest.mark.parametrize("eps,sigma", [(1.73, 1.0), (0.0, 1.0), (1.73, 0.25), (2.5, 4.0)])
def test_force_moment_form_equals_aij_form(oracle, eps, sigma):
    p = oracle.make_params(13, 11, epsilon=eps, sigma=sigma, G=-1.0)
    psi = _random_psi(13, 11, 3)
    Fx, Fy = oracle.force(p, psi)
    Ax, Ay = oracle.force(p, psi, aij=True)
    scale = max(np.abs(Fx).max(), np.abs(Fy).max())
    assert np.abs(Fx - Ax).max() < 1e-14 * scale
    assert np.abs(Fy - Ay).max() < 1e-14 * scale


def test_force_sums_to_zero_on_periodic_lattice(oracle):
    p = oracle.make_params(17, 12, epsilon=1.73, sigma=2.0)
    psi = _random_psi(17, 12, 4)
    Fx, Fy = oracle.force(p, psi)
    scale = np.abs(Fx).sum() + np.abs(Fy).sum()
    assert abs(Fx.sum()) < 1e-14 * scale and abs(Fy.sum()) < 1e-14 * scale


def test_force_zero_for_uniform_psi(oracle):
    p = oracle.make_params(8, 8, epsilon=1.73, sigma=0.5)
    Fx, Fy = oracle.force(p, np.full((8, 8), 0.7))
    assert np.abs(Fx).max() < 1e-16 and np.abs(Fy).max() < 1e-16


def test_shan_chen_special_case(oracle):
    # eps = 0, sigma = 1 is the Shan-Chen force (Eq. SCF), written here with np.roll.
    nx, ny = 15, 9
    psi = _random_psi(nx, ny, 5)
    G = -1.0
    p = oracle.make_params(nx, ny, epsilon=0.0, sigma=1.0, G=G)
    Fx, Fy = oracle.force(p, psi)
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    sx = np.zeros_like(psi)
    sy = np.zeros_like(psi)
    for i in range(9):
        cx, cy = int(C[i, 0]), int(C[i, 1])
        nb = np.roll(np.roll(psi, -cy, axis=0), -cx, axis=1)  # psi(x + c_i)
        sx += w[i] * nb * cx
        sy += w[i] * nb * cy
    assert np.allclose(Fx, -psi * 2 * G / CS2 * sx, atol=1e-15, rtol=0)
    assert np.allclose(Fy, -psi * 2 * G / CS2 * sy, atol=1e-15, rtol=0)


def test_force_depends_only_on_sign_of_G(oracle):
    # psi = sqrt((P - cs^2 rho)/G) scales as |G|^(-1/2) and F ~ G psi psi.
    nx, ny = 20, 16
    rho = W.smooth_random(nx, ny, 6, mean=0.15, amplitude=0.1)
    out = []
    for G in (-1.0, -7.5):
        p = W.params(nx, ny, tr=0.8)
        p["G"] = G
        P = oracle_params(oracle, p)
        f = oracle.init(P, rho)
        m = oracle.moments(P, f)
        out.append((m["Fx"], m["Fy"]))
    scale = np.abs(out[0][0]).max()
    assert np.abs(out[0][0] - out[1][0]).max() < 1e-13 * scale
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-13 * scale


def _spectral_derivative(f, ox, oy):
    """d^ox/dx^ox d^oy/dy^oy of a periodic field, exact for trig polynomials."""
    ny, nx = f.shape
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")
    return np.real(np.fft.ifft2(np.fft.fft2(f) * (1j * KX) ** ox * (1j * KY) ** oy))


@pytest.mark.parametrize("eps,sigma", [(1.73, 1.0), (1.73, 3.0), (0.0, 0.25)])
def test_force_continuum_limit(oracle, eps, sigma):
    # The discrete force approaches its continuum form, Eq. CFSCF for F^SC plus
    # Eqs. CCFT and SSTFT for F^(1), F^(2):
    #   F = -G (grad psi^2 + cs^2 psi grad Lap psi)
    #       - (3/4) eps cs^2 G (-2 d_b psi d_a d_b psi)
    #       + (sigma-1) cs^2 G (d_a psi Lap psi - d_b psi d_a d_b psi).
    # The first neglected terms are O(k^4) relative to the leading one, so the
    # relative error must fall ~16x per halving of k; a wrong coefficient or
    # sign leaves an O(k^2) error that falls only 4x.
    G = -1.0
    errs = []
    for n in (24, 48, 96):
        k = 2 * np.pi / n
        y, x = np.mgrid[0:n, 0:n].astype(float)
        psi = 1.0 + 0.3 * np.sin(k * x) + 0.2 * np.cos(k * (x + y) + 0.4) * np.sin(k * y + 0.4)
        d = lambda ox, oy: _spectral_derivative(psi, ox, oy)
        px, py = d(1, 0), d(0, 1)
        pxx, pxy, pyy = d(2, 0), d(1, 1), d(0, 2)
        lap = pxx + pyy
        lapx, lapy = d(3, 0) + d(1, 2), d(2, 1) + d(0, 3)
        Fsc = np.stack([-G * (2 * psi * px + CS2 * psi * lapx),
                        -G * (2 * psi * py + CS2 * psi * lapy)])
        F1 = np.stack([-2 * (px * pxx + py * pxy), -2 * (px * pxy + py * pyy)])
        F2 = np.stack([px * lap - (px * pxx + py * pxy), py * lap - (px * pxy + py * pyy)])
        Fc = Fsc - 0.75 * eps * CS2 * G * F1 + (sigma - 1) * CS2 * G * F2
        p = oracle.make_params(n, n, epsilon=eps, sigma=sigma, G=G)
        Fx, Fy = oracle.force(p, psi)
        errs.append(max(np.abs(Fx - Fc[0]).max(), np.abs(Fy - Fc[1]).max()) / np.abs(Fc).max())
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 12.0), (errs, ratios)


def test_alternative_trace_stencil(oracle):
    # m2_trace_alt replaces M2_bb by 2 cs^2 (M0 - psi) (stated after Eq. DFTCST);
    # only the F^(2) term changes, by (sigma-1) cs^2 G (M1_a/cs^2)(dT/cs^4).
    nx, ny = 12, 10
    psi = _random_psi(nx, ny, 7)
    eps, sigma, G = 1.73, 2.5, -1.0
    pd = oracle.make_params(nx, ny, epsilon=eps, sigma=sigma, G=G, m2_trace_alt=False)
    pa = oracle.make_params(nx, ny, epsilon=eps, sigma=sigma, G=G, m2_trace_alt=True)
    Fdx, Fdy = oracle.force(pd, psi)
    Fax, Fay = oracle.force(pa, psi)
    m = oracle.psi_moments(psi)
    dT = 2 * CS2 * (m["M0"] - psi) - (m["M2xx"] + m["M2yy"])
    assert np.abs(dT).max() > 1e-3  # the two stencils really differ on rough fields
    k = (sigma - 1) * CS2 * G / (CS2 * CS2 * CS2)
    assert np.allclose(Fax - Fdx, k * m["M1x"] * dT, atol=1e-14, rtol=0)
    assert np.allclose(Fay - Fdy, k * m["M1y"] * dT, atol=1e-14, rtol=0)
    # for a field whose fourth derivatives vanish on the stencil (a linear ramp
    # in y, constant in x, no wrap inside the interior) the two traces agree
    ramp = np.tile(0.5 + 0.01 * np.arange(ny, dtype=float)[:, None], (1, nx))
    m = oracle.psi_moments(ramp)
    inner = slice(1, ny - 1)
    tr_d = (m["M2xx"] + m["M2yy"])[inner]
    tr_a = (2 * CS2 * (m["M0"] - ramp))[inner]
    assert np.allclose(tr_d, tr_a, atol=1e-15)


def test_eos_and_psi_domain(oracle):
    p = oracle.make_params(4, 4, eos=(1, 1, 1, 1), T=0.8 * W.UNIT_CS_TC)
    rho = 0.2
    br = rho
    P = (rho * p.T * (1 + br + br**2 - br**3) / (1 - br) ** 3 - rho**2)
    assert abs(oracle.eos_pressure(p, rho) - P) < 1e-16
    assert abs(oracle.psi(p, rho) - math.sqrt((P - rho / 3) / -1.0)) < 1e-15
    for bad in (0.0, -0.1, 1.0, 1.5, float("nan")):
        with pytest.raises(oracle.OracleError):
            oracle.psi(p, bad)
    # above rho_max the radicand turns negative (G < 0 needs P < rho/3)
    with pytest.raises(oracle.OracleError):
        oracle.psi(p, 0.9)

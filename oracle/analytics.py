"""Macroscopic theory of the force-approach pseudopotential LBM, CPU FP64.

TEST INFRASTRUCTURE ONLY (part of the oracle).  These routines give what the
paper's theory predicts for the lattice runs, so that physics checks have an
expected value that does not come from any lattice code:

  * the Carnahan-Starling EOS (Eq. CSEOS) and its critical point;
  * Maxwell's equal-area coexistence (Eq. MLVDR);
  * the mechanical-equilibrium coexistence of a planar interface
    (Eqs. PGLDR, BPLP, BPVP) with eps = -2 A1/(A2 + A3);
  * the planar surface tension (Eqs. STDIM, STPI) by the paper's finite
    difference + Newton procedure (end of Sec. II.B) and, as a cross-check,
    by a first integral of Eq. PTNNPI;
  * Lamb's oscillation period of a 2D droplet (Eq. DOP).

For the proposed force the pressure-tensor coefficients are those of
Eq. PTIFT: A1 = -(3/4) eps cs^2, A2 + A3 = (3/2) cs^2, A3 = sigma cs^2.
Eq. STPI is printed without the factor G; since p_xx - p_yy = G A3 psi psi''
(Eqs. PTNNPI, PTTTPI), the factor is kept here, which makes gamma positive.
"""
import warnings
from dataclasses import dataclass

import numpy as np
from scipy import integrate, optimize
from scipy.linalg import solve_banded

CS2 = 1.0 / 3.0



def _quad(fn, a, b, epsrel):
    # quad's round-off notices at the requested relative accuracy are harmless
    # here: every pin taken from these routines has 4-5 significant digits.
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        return integrate.quad(fn, a, b, epsabs=0.0, epsrel=epsrel, limit=500)[0]


@dataclass(frozen=True)
class CarnahanStarling:
    """P = k [ c rho T (1 + b rho + (b rho)^2 - (b rho)^3)/(1 - b rho)^3 - a rho^2 ] (Eq. CSEOS)."""
    a: float
    b: float
    c: float
    k: float

    @property
    def rho_max(self):
        """Upper end of the density domain (packing limit b rho < 1)."""
        return 1.0 / self.b

    def P(self, rho, T):
        br = self.b * rho
        return self.k * (self.c * rho * T * (1 + br + br**2 - br**3) / (1 - br) ** 3
                         - self.a * rho**2)

    def dP(self, rho, T):
        # d/drho of rho*Z(b rho) with Z = (1 + e + e^2 - e^3)/(1 - e)^3 is
        # (1 + 4e + 4e^2 - 4e^3 + e^4)/(1 - e)^4, from the quotient rule.
        e = self.b * rho
        dz = (1 + 4 * e + 4 * e**2 - 4 * e**3 + e**4) / (1 - e) ** 4
        return self.k * (self.c * T * dz - 2 * self.a * rho)

    def d2P(self, rho, T):
        e = self.b * rho
        # derivative of (1 + 4e + 4e^2 - 4e^3 + e^4)/(1 - e)^4 with respect to e
        num = 1 + 4 * e + 4 * e**2 - 4 * e**3 + e**4
        dnum = 4 + 8 * e - 12 * e**2 + 4 * e**3
        dd = (dnum * (1 - e) + 4 * num) / (1 - e) ** 5
        return self.k * (self.c * T * self.b * dd - 2 * self.a)


# The equation of state of the paper's simulations (Sec. IV.A).
PAPER_EOS = CarnahanStarling(a=3.852462257, b=0.1304438842, c=2.785855166, k=0.01)
# Carnahan-Starling in the a = 1, b = 4, R = 1 convention of Yuan and Schaefer
# (eta = b rho / 4), which is Eq. CSEOS with a = b = c = k = 1.
UNIT_EOS = CarnahanStarling(a=1.0, b=1.0, c=1.0, k=1.0)


def critical_point(eos: CarnahanStarling):
    """(rho_c, T_c, p_c) where dP/drho = d2P/drho2 = 0."""
    def T_on_spinodal(rho):  # dP/drho = 0 solved for T
        e = eos.b * rho
        dz = (1 + 4 * e + 4 * e**2 - 4 * e**3 + e**4) / (1 - e) ** 4
        return 2 * eos.a * rho / (eos.c * dz)

    # the critical point is the maximum of the spinodal temperature
    res = optimize.minimize_scalar(lambda r: -T_on_spinodal(r),
                                   bounds=(1e-6 / eos.b, 0.9 / eos.b), method="bounded",
                                   options={"xatol": 1e-13 / eos.b})
    # refine: at the critical point d2P/drho2 = 0 with T = T_spinodal(rho)
    f = lambda r: eos.d2P(r, T_on_spinodal(r))
    lo, hi = res.x * 0.9, res.x * 1.1
    rho_c = optimize.brentq(f, lo, hi, xtol=1e-15, rtol=1e-15)
    T_c = T_on_spinodal(rho_c)
    return rho_c, T_c, float(eos.P(rho_c, T_c))


def spinodals(eos: CarnahanStarling, T):
    """Densities where dP/drho = 0 on either side of the unstable branch.  An
    equation of state other than Carnahan-Starling supplies its own (any
    object with P, dP, rho_max and spinodals(T) can be passed to the
    coexistence routines below)."""
    if not isinstance(eos, CarnahanStarling):
        return eos.spinodals(T)
    rho_c, T_c, _ = critical_point(eos)
    if T >= T_c:
        raise ValueError("no two-phase region above T_c")
    f = lambda r: eos.dP(r, T)
    r1 = optimize.brentq(f, 1e-12 / eos.b, rho_c, xtol=1e-15)
    r2 = optimize.brentq(f, rho_c, (1 - 1e-9) / eos.b, xtol=1e-15)
    return r1, r2


def _coexistence(eos, T, area):
    """Solve P(rho_g) = P(rho_l) = p0 and area(p0, rho_g, rho_l) = 0 for p0."""
    s1, s2 = spinodals(eos, T)
    p_hi = eos.P(s1, T)
    p_lo = max(eos.P(s2, T), 1e-300)

    def roots(p0):
        rg = optimize.brentq(lambda r: eos.P(r, T) - p0, 1e-300, s1, xtol=1e-300, rtol=1e-15)
        rl = optimize.brentq(lambda r: eos.P(r, T) - p0, s2, (1 - 1e-12) * eos.rho_max,
                             xtol=1e-300, rtol=1e-15)
        return rg, rl

    def g(p0):
        rg, rl = roots(p0)
        return area(p0, rg, rl)

    eps = 1e-12 * (p_hi - p_lo)
    a, b = p_lo + eps, p_hi - eps
    if g(a) * g(b) > 0:
        raise ValueError("no coexistence pressure between the spinodal pressures")
    p0 = optimize.brentq(g, a, b, xtol=1e-300, rtol=1e-15)
    rg, rl = roots(p0)
    return rg, rl, p0


def maxwell(eos: CarnahanStarling, T):
    """Maxwell equal-area coexistence (Eq. MLVDR): int (p0 - P) drho / rho^2 = 0."""
    def area(p0, rg, rl):
        return _quad(lambda r: (p0 - eos.P(r, T)) / r**2, rg, rl, 1e-11)
    return _coexistence(eos, T, area)


def psi_of_rho(eos, T, rho, G=-1.0):
    """Eq. DED: psi = sqrt((P - cs^2 rho)/G)."""
    return np.sqrt((eos.P(rho, T) - CS2 * rho) / G)


def dpsi_drho(eos, T, rho, G=-1.0):
    return (eos.dP(rho, T) - CS2) / (2 * G * psi_of_rho(eos, T, rho, G))


def mechanical_coexistence(eos: CarnahanStarling, T, eps, G=-1.0):
    """Planar-interface coexistence of the pseudopotential method (Eq. PGLDR):
    int (p0 - cs^2 rho - G psi^2) psi_dot / psi^(1+eps) drho = 0, where
    cs^2 rho + G psi^2 = P_EOS by Eq. DED."""
    def area(p0, rg, rl):
        fn = lambda r: ((p0 - eos.P(r, T)) * dpsi_drho(eos, T, r, G)
                        / psi_of_rho(eos, T, r, G) ** (1 + eps))
        return _quad(fn, rg, rl, 1e-11)
    return _coexistence(eos, T, area)


def force_coefficients(eps, sigma):
    """A1, A2 + A3 and A3 of the pressure tensor realised by Eq. IFT (Eq. PTIFT)."""
    return -0.75 * eps * CS2, 1.5 * CS2, sigma * CS2


def planar_profile_fd(eos, T, eps, L=30.0, dx=0.1, G=-1.0, tol=1e-12, max_iter=400):
    """Density profile of a planar interface: Eq. PTNNPI with p_xx = p0, second-order
    central differences on [0, L] and Dirichlet densities from Eq. PGLDR at the
    ends, solved by Newton-Raphson (end of Sec. II.B).  Returns x, rho, psi, p0."""
    rg, rl, p0 = mechanical_coexistence(eos, T, eps, G)
    A1, B, _ = force_coefficients(eps, 1.0)
    n = int(round(L / dx))
    x = np.linspace(0.0, L, n + 1)
    h = x[1] - x[0]
    rho = 0.5 * (rl + rg) + 0.5 * (rl - rg) * np.tanh((x - L / 2) / 2.0)
    rho[0], rho[-1] = rg, rl

    def residual(r):
        psi = psi_of_rho(eos, T, r, G)
        d1 = (psi[2:] - psi[:-2]) / (2 * h)
        d2 = (psi[2:] - 2 * psi[1:-1] + psi[:-2]) / h**2
        pm = r[1:-1]
        return (CS2 * pm + G * psi[1:-1] ** 2 + G * (A1 * d1**2 + B * psi[1:-1] * d2) - p0,
                psi, d1, d2)

    for _ in range(max_iter):
        res, psi, d1, d2 = residual(rho)
        if np.max(np.abs(res)) < tol:
            break
        dpsi = dpsi_drho(eos, T, rho, G)
        # Jacobian of res_j with respect to rho_{j-1}, rho_j, rho_{j+1} (tridiagonal)
        diag = (CS2 + 2 * G * psi[1:-1] * dpsi[1:-1]
                + G * B * dpsi[1:-1] * (d2 - 2 * psi[1:-1] / h**2))
        upper = G * (A1 * 2 * d1 / (2 * h) + B * psi[1:-1] / h**2) * dpsi[2:]
        lower = G * (-A1 * 2 * d1 / (2 * h) + B * psi[1:-1] / h**2) * dpsi[:-2]
        m = n - 1
        ab = np.zeros((3, m))
        ab[0, 1:] = upper[:-1]
        ab[1, :] = diag
        ab[2, :-1] = lower[1:]
        delta = solve_banded((1, 1), ab, -res)
        # damp so the iterate stays inside (rho_g/2, 1/b)
        lam = 1.0
        while lam > 1e-6:
            trial = rho.copy()
            trial[1:-1] += lam * delta
            if np.all(trial > 0) and np.all(eos.b * trial < 1) and np.all(
                    (eos.P(trial, T) - CS2 * trial) / G > 0):
                break
            lam *= 0.5
        rho = trial
    else:
        raise RuntimeError("planar profile Newton did not converge")
    return x, rho, psi_of_rho(eos, T, rho, G), p0


def planar_surface_tension_fd(eos, T, eps, sigma, L=30.0, dx=0.1, G=-1.0):
    """gamma_pi = int G A3 psi psi'' dx over the finite-difference profile (Eq. STPI)."""
    x, rho, psi, _ = planar_profile_fd(eos, T, eps, L, dx, G)
    h = x[1] - x[0]
    _, _, A3 = force_coefficients(eps, sigma)
    d2 = (psi[2:] - 2 * psi[1:-1] + psi[:-2]) / h**2
    return float(G * A3 * np.sum(psi[1:-1] * d2) * h)


def planar_surface_tension_quad(eos, T, eps, sigma, G=-1.0):
    """gamma_pi from a first integral of Eq. PTNNPI.  With y(psi) = psi'^2 the
    balance p_xx = p0 becomes A1 y + (B/2) psi dy/dpsi = (p0 - P)/G, whose
    solution with y(psi_g) = 0 is
        y(psi) = psi^eps (2/(G B)) int_{psi_g}^{psi} (p0 - P) s^(-1-eps) ds,
    and gamma_pi = G A3 int psi psi'' dx = -G A3 int sqrt(y) dpsi."""
    rg, rl, p0 = mechanical_coexistence(eos, T, eps, G)
    _, B, A3 = force_coefficients(eps, sigma)

    def inner(rho):
        fn = lambda r: ((p0 - eos.P(r, T)) * dpsi_drho(eos, T, r, G)
                        / psi_of_rho(eos, T, r, G) ** (1 + eps))
        val = _quad(fn, rg, rho, 1e-11)
        return psi_of_rho(eos, T, rho, G) ** eps * 2.0 / (G * B) * val

    outer = lambda r: np.sqrt(max(inner(r), 0.0)) * dpsi_drho(eos, T, r, G)
    val = _quad(outer, rg, rl, 1e-10)
    return float(-G * A3 * val)


def lamb_period(gamma, rho_l, R_max, R_min, n=2):
    """Eq. DOP: T_a = 2 pi [ n (n^2 - 1) gamma / (rho_l R_m^3) ]^(-1/2), R_m = sqrt(R_max R_min)."""
    Rm = np.sqrt(R_max * R_min)
    return float(2 * np.pi * (n * (n**2 - 1) * gamma / (rho_l * Rm**3)) ** -0.5)


def fit_epsilon(eos, T, lo=1.0, hi=2.5, G=-1.0):
    """eps whose planar coexistence (Eq. PGLDR) gives Maxwell's liquid density
    (the consistency condition of Eq. CTC, imposed at one temperature).  Both
    coexistence densities are roots of P = p0, so matching the liquid density
    matches p0 and the gas density too.  The bracket is scanned first, since
    Eq. PGLDR has no solution for some eps.  For an equation of state that
    satisfies Eq. CTC exactly with some eps0 the result is eps0; for the
    Carnahan-Starling sets it is 1.89-1.93 (paper's constants) and 1.64-1.76
    (a = b = c = k = 1) over T_r = 0.6 .. 0.9.  The paper's 1.73 was found by
    adjusting lattice runs, not from Eq. PGLDR."""
    _, rl_m, _ = maxwell(eos, T)

    def diff(e):
        try:
            return mechanical_coexistence(eos, T, e, G)[1] - rl_m
        except ValueError:
            return None

    grid = np.linspace(lo, hi, 31)
    vals = [diff(e) for e in grid]
    for (e0, v0), (e1, v1) in zip(zip(grid, vals), zip(grid[1:], vals[1:])):
        if v0 is not None and v1 is not None and v0 * v1 <= 0:
            return optimize.brentq(diff, e0, e1, xtol=1e-10)
    raise ValueError("no eps in the bracket matches the Maxwell liquid density")

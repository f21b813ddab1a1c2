"""Small helpers shared by the tests: parameter conversion and measurements.

Nothing here computes any part of the lattice update."""
import numpy as np


def oracle_params(oracle, p):
    """Oracle parameter struct from a workloads.params() dictionary."""
    return oracle.make_params(p["nx"], p["ny"], tau=p["tau"], G=p["G"], epsilon=p["epsilon"],
                              sigma=p["sigma"],
                              eos=(p["eos_a"], p["eos_b"], p["eos_c"], p["eos_k"]), T=p["T"],
                              force_on=p["force_on"], m2_trace_alt=p["m2_trace_alt"],
                              storage=p.get("storage", 0), rho_ref=p.get("rho_ref", 0.0),
                              collision=p.get("collision", 0),
                              mrt=tuple(p.get(k, 1.0) for k in ("tau_rho", "tau_e", "tau_zeta",
                                                                "tau_j", "tau_q")))


def slab_bulk(rho):
    """Bulk liquid and gas densities of a slab occupying the middle half in x:
    means over the cells at least nx/8 away from both interfaces."""
    row = rho.mean(axis=0)
    n = row.size
    liq = row[3 * n // 8:5 * n // 8].mean()
    gas = np.r_[row[:n // 8], row[n - n // 8:]].mean()
    return float(liq), float(gas)


def droplet_measure(rho, outer_margin):
    """Radius at rho_m = (max+min)/2 from the four axis rays (linear
    interpolation, averaged), mean density inside R/2 and beyond R + margin."""
    ny, nx = rho.shape
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx]
    r = np.hypot(x - cx, y - cy)
    rm = 0.5 * (rho.max() + rho.min())
    row = rho[ny // 2 - 1:ny // 2 + 1, :].mean(0)
    col = rho[:, nx // 2 - 1:nx // 2 + 1].mean(1)
    radii = []
    for prof in (row[nx // 2:], row[:nx // 2][::-1], col[ny // 2:], col[:ny // 2][::-1]):
        d = np.arange(prof.size) + 0.5
        j = int(np.where(prof < rm)[0][0])
        radii.append(d[j - 1] + (prof[j - 1] - rm) / (prof[j - 1] - prof[j]))
    R = float(np.mean(radii))
    return R, float(rho[r < R / 2].mean()), float(rho[r > R + outer_margin].mean())


def x_extent(band, rho_m):
    """Half-length of the liquid region along +x through the centre of an
    nx-wide lattice with an even number of rows: band holds the two rows next
    to y0 = (ny-1)/2; returns the distance from x0 = (nx-1)/2 to where their
    mean density first falls below rho_m (linear interpolation between cell
    centres)."""
    nx = band.shape[1]
    row = band.mean(0)[nx // 2:]
    d = np.arange(row.size) + (nx // 2 - (nx - 1) / 2.0)
    j = int(np.where(row < rho_m)[0][0])
    return float(d[j - 1] + (row[j - 1] - rho_m) / (row[j - 1] - row[j]) * (d[j] - d[j - 1]))


def fit_damped_period(t, r):
    """Period T of r(t) = c + A exp(-lam t) cos(2 pi t / T + phi), least squares
    over all samples.  The starting guess takes T as twice the time of the
    first minimum."""
    from scipy.optimize import curve_fit
    t = np.asarray(t, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    T0 = 2.0 * t[int(np.argmin(r[: len(r) * 3 // 4]))]
    c0 = 0.5 * (r.max() + r.min())

    def model(tt, c, A, lam, T, phi):
        return c + A * np.exp(-lam * tt) * np.cos(2 * np.pi * tt / T + phi)

    p0 = (c0, r[0] - c0, 1.0 / t[-1], T0, 0.0)
    popt, _ = curve_fit(model, t, r, p0=p0, maxfev=20000)
    return float(abs(popt[3])), popt

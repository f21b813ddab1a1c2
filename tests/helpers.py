"""Small helpers shared by the tests: parameter conversion and measurements.

Nothing here computes any part of the lattice update."""
import numpy as np


def oracle_params(oracle, p):
    """Oracle parameter struct from a workloads.params() dictionary."""
    return oracle.make_params(p["nx"], p["ny"], tau=p["tau"], G=p["G"], epsilon=p["epsilon"],
                              sigma=p["sigma"],
                              eos=(p["eos_a"], p["eos_b"], p["eos_c"], p["eos_k"]), T=p["T"],
                              force_on=p["force_on"], m2_trace_alt=p["m2_trace_alt"],
                              storage=p.get("storage", 0), rho_ref=p.get("rho_ref", 0.0))


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

"""Seeded synthetic inputs for the D2Q9 pseudopotential lattice update.

This module generates initial density fields and parameter sets.  The tests
feed the same arrays to the HIP library and to the CPU oracle, and the
benchmark uses them to build its workload.  It holds none of the method's
arithmetic: no equilibrium, force, collision or streaming, only the initial
shapes of Sec. IV (Eqs. ISD and REL) and seeded noise.

Equation of state.  A Carnahan-Starling EOS in the "a = 1, b = 4, R = 1"
convention of Yuan and Schaefer (packing fraction b rho / 4) is Eq. CSEOS with
a = b = c = k = 1 (UNIT_CS).  The paper's own set (Sec. IV.A) is PAPER_CS,
whose critical point is rho_c = T_c = 1, so that its T is the reduced
temperature.

Coexistence estimates.  Initial liquid and gas densities are the Maxwell
equal-area values (Eq. MLVDR) of UNIT_CS, tabulated below at reduced
temperatures 0.50, 0.55, ..., 0.95 and interpolated in between (log-linear for
the gas, linear for the liquid).  They are only starting estimates; the lattice
relaxes to its own coexistence.
"""
import math

import numpy as np

UNIT_CS = {"eos_a": 1.0, "eos_b": 1.0, "eos_c": 1.0, "eos_k": 1.0}
PAPER_CS = {"eos_a": 3.852462257, "eos_b": 0.1304438842, "eos_c": 2.785855166, "eos_k": 0.01}

# Critical temperature and density of UNIT_CS (dP/drho = d2P/drho2 = 0).
UNIT_CS_TC = 0.09432870313372377
UNIT_CS_RHOC = 0.13044388419245395
PAPER_CS_TC = 1.0

# Maxwell coexistence of UNIT_CS: reduced temperature -> (rho_gas, rho_liquid).
UNIT_CS_MAXWELL = {
    0.50: (6.265678136210e-04, 4.540784256808e-01),
    0.55: (1.509384291077e-03, 4.300282945352e-01),
    0.60: (3.081458538701e-03, 4.062041397690e-01),
    0.65: (5.586886971204e-03, 3.823354103970e-01),
    0.70: (9.294146214955e-03, 3.581309411885e-01),
    0.75: (1.452608460572e-02, 3.332415985387e-01),
    0.80: (2.172324341156e-02, 3.071956823671e-01),
    0.85: (3.158177949692e-02, 2.792620942592e-01),
    0.90: (4.542119805617e-02, 2.480842412089e-01),
    0.95: (6.661162921133e-02, 2.102542248280e-01),
}

# The paper's Maxwell values at T_r = 0.8 (Sec. IV.B, caption of Table DVT).
PAPER_CS_MAXWELL = {0.80: (0.1665, 2.3550)}


def unit_cs_coexistence(tr: float):
    """Maxwell (rho_gas, rho_liquid) estimate of UNIT_CS at reduced temperature tr."""
    keys = sorted(UNIT_CS_MAXWELL)
    if not keys[0] <= tr <= keys[-1]:
        raise ValueError(f"reduced temperature {tr} outside [{keys[0]}, {keys[-1]}]")
    for lo, hi in zip(keys, keys[1:]):
        if lo <= tr <= hi:
            s = (tr - lo) / (hi - lo)
            g0, l0 = UNIT_CS_MAXWELL[lo]
            g1, l1 = UNIT_CS_MAXWELL[hi]
            return math.exp((1 - s) * math.log(g0) + s * math.log(g1)), (1 - s) * l0 + s * l1
    return UNIT_CS_MAXWELL[keys[-1]]


# f16l: binary16 deviations from w_i times a per-cell FP32 reference density
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "f16l": 3}


COLLISION = {"bgk": 0, "mrt": 1}


def params(nx, ny, tr=0.8, tau=1.0, G=-1.0, epsilon=1.73, sigma=1.0, eos="unit",
           force_on=True, m2_trace_alt=False, storage="f64", rho_ref=0.0, collision="bgk",
           mrt=(1.0, 1.0, 1.0, 1.0, 1.0)):
    """A parameter dictionary in the field names of the library's parameter block.
    storage is "f64", "f32" or "f16" (the last two store deviations from
    w_i rho_ref).  collision is "bgk" or "mrt"; mrt holds the MRT relaxation
    times (tau_rho, tau_e, tau_zeta, tau_j, tau_q), the stress rows relaxing
    with tau."""
    if eos == "unit":
        p = dict(UNIT_CS)
        T = tr * UNIT_CS_TC
    elif eos == "paper":
        p = dict(PAPER_CS)
        T = tr * PAPER_CS_TC
    else:
        raise ValueError(eos)
    p.update(nx=int(nx), ny=int(ny), tau=float(tau), G=float(G), epsilon=float(epsilon),
             sigma=float(sigma), T=float(T), force_on=bool(force_on),
             m2_trace_alt=bool(m2_trace_alt), storage=STORAGE[storage], rho_ref=float(rho_ref),
             collision=COLLISION[collision])
    p.update(zip(("tau_rho", "tau_e", "tau_zeta", "tau_j", "tau_q"), (float(v) for v in mrt)))
    return p


def shift_reference(rho0, storage):
    """Reference density rho_ref of the shifted storage modes.  FP32: the mean
    density.  FP16: the smallest density, so that the gas phase of a
    two-phase field is stored as small deviations (binary16 keeps 11
    significant bits of each deviation; with the mean as reference the gas
    populations would be stored as deviations several times larger than
    themselves).  FP64 storage and the per-cell mode take no global reference."""
    if storage in ("f64", 0, "f16l", 3):
        return 0.0
    if storage in ("f32", 1):
        return float(np.mean(rho0))
    return float(np.min(rho0))


def noise(shape, seed, amplitude=1e-3):
    """Additive uniform noise U(-amplitude, amplitude) from NumPy's PCG64."""
    return np.random.default_rng(seed).uniform(-amplitude, amplitude, size=shape)


def droplet(nx, ny, radius, rho_l, rho_g, width=2.0, center=None):
    """Circular droplet, Eq. ISD: rho = (rho_l + rho_g)/2 - (rho_l - rho_g)/2 tanh(2 (R - R0)/W),
    with R measured from the domain centre ((nx-1)/2, (ny-1)/2) in cell units."""
    x0, y0 = ((nx - 1) / 2.0, (ny - 1) / 2.0) if center is None else center
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - x0) ** 2 + (y - y0) ** 2)
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2.0 * (r - radius) / width)


def ellipse(nx, ny, r_max, r_min, rho_l, rho_g, width=2.0):
    """Elliptical droplet, Eqs. ISD and REL: R0(theta) = R_min / sqrt(1 - (e cos theta)^2),
    e = sqrt(1 - (R_min/R_max)^2), major axis along x.  theta uses atan2, which
    leaves R0 unchanged (it depends only on cos^2 theta) and is defined at x = x0."""
    x0, y0 = (nx - 1) / 2.0, (ny - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - x0) ** 2 + (y - y0) ** 2)
    theta = np.arctan2(y - y0, x - x0)
    e = math.sqrt(1.0 - (r_min / r_max) ** 2)
    r0 = r_min / np.sqrt(1.0 - (e * np.cos(theta)) ** 2)
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh(2.0 * (r - r0) / width)


def slab(nx, ny, rho_l, rho_g, width=2.0):
    """Flat liquid slab in the middle half of the domain, uniform in y:
    rho = rho_g + (rho_l - rho_g)/2 [tanh(2 (x - x1)/W) - tanh(2 (x - x2)/W)],
    x1 = nx/4 - 1/2, x2 = 3 nx/4 - 1/2."""
    x = np.arange(nx, dtype=np.float64)
    x1, x2 = nx / 4.0 - 0.5, 3.0 * nx / 4.0 - 0.5
    row = rho_g + 0.5 * (rho_l - rho_g) * (np.tanh(2.0 * (x - x1) / width)
                                          - np.tanh(2.0 * (x - x2) / width))
    return np.ascontiguousarray(np.broadcast_to(row, (ny, nx)))


def smooth_random(nx, ny, seed, mean, amplitude, modes=4):
    """A smooth periodic random field: a few low Fourier modes with seeded phases.
    Used for single-step parity on fields without interfaces."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    out = np.full((ny, nx), float(mean))
    for _ in range(modes):
        kx, ky = rng.integers(0, 3, size=2)
        if kx == 0 and ky == 0:
            kx = 1
        ph = rng.uniform(0, 2 * np.pi)
        a = rng.uniform(0.3, 1.0)
        out += amplitude * a / modes * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
    return out


# ---- named workloads (sizes and recipes of the synthetic configurations) ----

def droplet_64(seed=1):
    """64 x 64 periodic droplet, R0 = 16, W = 2, T_r = 0.8, tau = 1, UNIT_CS,
    Maxwell densities, U(+-1e-3) noise.  Returns (params, rho0)."""
    p = params(64, 64, tr=0.8, tau=1.0)
    rg, rl = unit_cs_coexistence(0.8)
    rho0 = droplet(64, 64, 16.0, rl, rg, 2.0) + noise((64, 64), seed)
    return p, rho0


def slab_case(n=2048, ny=None, tr=0.8, seed=None, tau=1.0):
    """n x ny periodic flat slab (middle half liquid), W = 2, UNIT_CS at reduced
    temperature tr, Maxwell densities, U(+-1e-3) noise.  The default seeds are
    2, 3, 4, 5 for T_r = 0.6, 0.7, 0.8, 0.9.  Returns (params, rho0)."""
    ny = n if ny is None else ny
    if seed is None:
        seed = {0.6: 2, 0.7: 3, 0.8: 4, 0.9: 5}.get(round(tr, 2), 2)
    p = params(n, ny, tr=tr, tau=tau)
    rg, rl = unit_cs_coexistence(tr)
    rho0 = slab(n, ny, rl, rg, 2.0) + noise((ny, n), seed)
    return p, rho0


def ellipse_case(n=1024, tr=0.7, tau=1.0, seed=8, r_max=160.0, r_min=120.0):
    """n x n periodic elliptical droplet (semi-axes r_max along x, r_min along y),
    W = 2, UNIT_CS at reduced temperature tr, U(+-1e-3) noise."""
    p = params(n, n, tr=tr, tau=tau)
    rg, rl = unit_cs_coexistence(tr)
    rho0 = ellipse(n, n, r_max, r_min, rl, rg, 2.0) + noise((n, n), seed)
    return p, rho0


def batch_case(count=256, seed=6, storage="f32", side_range=(64, 512)):
    """A batch of independent square droplet lattices: side = round(exp U(ln 64,
    ln 512)), T_r ~ U[0.55, 0.95], sigma ~ U[1/8, 4] (the range of Table DVT),
    R0 = U[0.15, 0.35] side, W = 2, tau = 1, eps = 1.73, U(+-1e-3) noise, the
    given storage.  Returns a list of (params, rho0)."""
    rng = np.random.default_rng(seed)
    lo, hi = side_range
    out = []
    for k in range(count):
        side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        tr = float(rng.uniform(0.55, 0.95))
        sigma = float(rng.uniform(0.125, 4.0))
        r0 = float(rng.uniform(0.15, 0.35)) * side
        p = params(side, side, tr=tr, tau=1.0, sigma=sigma, storage=storage)
        rg, rl = unit_cs_coexistence(tr)
        rho0 = droplet(side, side, r0, rl, rg, 2.0) + noise((side, side), seed * 100003 + k)
        p["rho_ref"] = shift_reference(rho0, storage)
        out.append((p, rho0))
    return out


def serve_case(count=64, seed=7, storage="f32", side_range=(64, 1024), steps_range=(2000, 50000)):
    """A stream of independent jobs: square lattices with side = round(exp
    U(ln 64, ln 1024)), steps ~ U{2000..50000}, a droplet (R0 = U[0.15, 0.35]
    side) or a flat slab with equal odds, T_r ~ U[0.55, 0.95], sigma ~ U[1/8, 4],
    tau = 1, eps = 1.73, W = 2, U(+-1e-3) noise.  Returns [(params, rho0, steps)]."""
    rng = np.random.default_rng(seed)
    lo, hi = side_range
    out = []
    for k in range(count):
        side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        nsteps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        tr = float(rng.uniform(0.55, 0.95))
        sigma = float(rng.uniform(0.125, 4.0))
        rg, rl = unit_cs_coexistence(tr)
        if rng.random() < 0.5:
            rho0 = droplet(side, side, float(rng.uniform(0.15, 0.35)) * side, rl, rg, 2.0)
        else:
            rho0 = slab(side, side, rl, rg, 2.0)
        rho0 = rho0 + noise((side, side), seed * 100003 + k)
        p = params(side, side, tr=tr, tau=1.0, sigma=sigma, storage=storage)
        p["rho_ref"] = shift_reference(rho0, storage)
        out.append((p, rho0, nsteps))
    return out


def poisson_arrivals(count, rate, seed=7):
    """Arrival times (seconds from 0) of a Poisson process of the given rate:
    cumulative sums of exponential gaps, the first job at 0."""
    gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, size=count)
    gaps[0] = 0.0
    return np.cumsum(gaps)

"""Shared pieces of the GPU tests: running the same seeded case through the
HIP library (through its C ABI) and through the CPU oracle, and the per-field
normwise comparison.

Tolerance.  Parity is measured per field and normwise, because a relative
error is ill-posed where u ~ 0:
    ||d rho||_inf / ||rho||_inf,  ||d(rho u)||_inf / (||rho||_inf c_s),
    ||d f||_inf / ||f||_inf
must each stay below PARITY_TOL = 1e-12 (FP64).  The two sides round
differently (the HIP compiler contracts multiply-adds into FMAs and the
kernel folds c_s^2 into its coefficients; the oracle keeps every operation
separate), so they agree to a few ulps per step, not bitwise."""
import sys

import numpy as np
import torch

PARITY_TOL = 1e-12
CS = 1.0 / np.sqrt(3.0)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_lattice(p, rho0, ux0=None, uy0=None, launch=None, fusion=None):
    """A lattice on the GPU.  launch = (block_x, seg_rows) selects single steps
    in that shape; fusion = (steps, block_x, seg_rows) the steps per pass and
    the two-step shape.  Neither: the library's defaults."""
    from paper_2003_07968_amd import lbm
    lat = lbm.Lattice(p, rho0, ux0, uy0)
    if launch is not None:
        lat.set_fusion(1)
        lat.set_launch(*launch)
    if fusion is not None:
        lat.set_fusion(*fusion)
    return lat


def gpu_state(lat):
    m = {k: v.cpu().numpy() for k, v in lat.moments().items()}
    m["f"] = lat.populations().cpu().numpy()
    return m


def oracle_state(oracle, P, f):
    m = oracle.moments(P, f)
    m["f"] = f.copy()
    return m


def parity_errors(g, o):
    rho_n = np.abs(o["rho"]).max()
    e_rho = np.abs(g["rho"] - o["rho"]).max() / rho_n
    e_mx = np.abs(g["rho"] * g["ux"] - o["rho"] * o["ux"]).max() / (rho_n * CS)
    e_my = np.abs(g["rho"] * g["uy"] - o["rho"] * o["uy"]).max() / (rho_n * CS)
    e_f = np.abs(g["f"] - o["f"]).max() / np.abs(o["f"]).max()
    return {"rho": e_rho, "mom": max(e_mx, e_my), "f": e_f}


def assert_parity(g, o, tol=PARITY_TOL, what=""):
    errs = parity_errors(g, o)
    log(f"  parity {what}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, f"{what}: {k} error {v:.3e} > {tol:.1e}"
    return errs


def require_gpu():
    assert torch.cuda.is_available(), "these tests need the MI355X"

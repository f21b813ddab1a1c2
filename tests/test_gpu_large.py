"""Large lattices, beyond what the CPU oracle steps in seconds: 8192 x 8192
(67 M cells; 9.7 GB of FP64 populations) in the library's default launch
(two steps per pass, the benchmarked path) and with single steps.

Sampled parity: f(t + s) of sampled cells against the oracle stepping the
neighbourhood of each cell s times, taken from the GPU's f(t) as a small
periodic lattice.  One update of a cell depends only on the cells within two
of it (the force of its neighbours needs psi one cell further), so s steps
depend on the cells within 2 s: the centre of a (4 s + 1)-square patch is the
exact oracle result for the large lattice (5 x 5 for one step, 9 x 9 for one
two-step pass).  The samples include lattice edges and the first and last
columns and rows of strips and segments of the launch.  Conservation of mass
and momentum holds at any size and is checked over the whole lattice."""
import numpy as np
import pytest
import torch

from paper_2003_07968_amd import workloads as W

from .gpu_common import CS, gpu_lattice, log, require_gpu
from .helpers import oracle_params

pytestmark = pytest.mark.gpu

N = 8192
TOL = {"f64": 1e-12, "f32": 1e-5}   # per cell, max |df| / max |f| of the cell


def _samples(launch, halo, rng):
    bx, rows, _ = launch
    width = (bx - 2 * halo) // 16 * 16
    xs = [0, 1, N - 2, N - 1, width - 1, width, 2 * width - 1, 2 * width]
    ys = [0, 1, N - 2, N - 1, rows - 1, rows, 5 * rows - 1, 5 * rows]
    cells = [(x, y) for x in xs for y in ys[:4]] + [(x, y) for x in xs[:4] for y in ys[4:]]
    cells += [tuple(int(v) for v in rng.integers(0, N, size=2)) for _ in range(32)]
    return cells


@pytest.mark.parametrize("steps", [2, 1])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_sampled_parity_and_conservation_8192(oracle, storage, steps):
    require_gpu()
    rng = np.random.default_rng(40)
    rg, rl = W.unit_cs_coexistence(0.8)
    rho0 = W.smooth_random(N, N, 41, mean=0.5 * (rg + rl), amplitude=0.45 * (rl - rg), modes=6)
    rho0 += W.noise((N, N), 42)
    p = W.params(N, N, tr=0.8, storage=storage)
    p["rho_ref"] = W.shift_reference(rho0, storage)
    lat = gpu_lattice(p, rho0, fusion=(steps,))
    assert lat.fusion() == steps
    launch = lat.launch()
    log(f"case {storage} {N}x{N}, {steps} step(s) per pass, launch {launch}")
    d0 = lat.diagnostics()
    lat.step(4)
    cells = _samples(launch, 3 if steps == 2 else 1, rng)
    f = lat.populations()
    r = 2 * steps
    idx = np.arange(-r, r + 1)
    patches = []
    for x, y in cells:
        ys = torch.as_tensor((y + idx) % N, device=f.device)
        xs = torch.as_tensor((x + idx) % N, device=f.device)
        patches.append(f[:, ys][:, :, xs].cpu().numpy())
    del f
    lat.step(steps)  # one pass
    f1 = lat.populations()
    got = [f1[:, y, x].cpu().numpy() for x, y in cells]
    del f1
    q = dict(p)
    q["nx"] = q["ny"] = 2 * r + 1
    Pp = oracle_params(oracle, q)
    worst = 0.0
    for (x, y), patch, g in zip(cells, patches, got):
        h = np.ascontiguousarray(patch)
        oracle.step(Pp, h, steps)
        err = np.abs(g - h[:, r, r]).max() / np.abs(h[:, r, r]).max()
        worst = max(worst, err)
        assert err <= TOL[storage], (x, y, err)
    d1 = lat.diagnostics()
    lat.sync()
    dm = abs(d1["mass"] / d0["mass"] - 1)
    mom = max(abs(d1["mom_x"]), abs(d1["mom_y"])) / (d0["mass"] * CS)
    log(f"  {len(cells)} sampled cells, worst {worst:.2e}; mass {dm:.1e}, momentum {mom:.1e}")
    assert dm < (1e-12 if storage == "f64" else 1e-5)
    assert mom < (1e-12 if storage == "f64" else 1e-5)

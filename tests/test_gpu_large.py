"""Large lattices, beyond what the CPU oracle steps in seconds: 8192 x 8192
(67 M cells; 9.7 GB of FP64 populations) in the library's default launch
shape.

Sampled parity: f(t + 1) of sampled cells against the oracle stepping the
5 x 5 neighbourhood of each cell, taken from the GPU's f(t) as a periodic
5 x 5 lattice.  The update of a cell depends only on the cells within two of
it (the force of its neighbours needs psi one cell further), so the centre of
the patch is the exact oracle update of the large lattice.  The samples
include lattice edges and the first and last columns and rows of strips and
segments of the launch.  Conservation of mass and momentum holds at any size
and is checked over the whole lattice."""
import numpy as np
import pytest
import torch

from paper_2003_07968_amd import workloads as W

from .gpu_common import CS, gpu_lattice, log, require_gpu
from .helpers import oracle_params

pytestmark = pytest.mark.gpu

N = 8192
TOL = {"f64": 1e-12, "f32": 1e-5}   # per cell, max |df| / max |f| of the cell


def _samples(launch, rng):
    bx, rows, _ = launch
    width = (bx - 2) // 16 * 16
    xs = [0, 1, N - 2, N - 1, width - 1, width, 2 * width - 1, 2 * width]
    ys = [0, 1, N - 2, N - 1, rows - 1, rows, 5 * rows - 1, 5 * rows]
    cells = [(x, y) for x in xs for y in ys[:4]] + [(x, y) for x in xs[:4] for y in ys[4:]]
    cells += [tuple(int(v) for v in rng.integers(0, N, size=2)) for _ in range(32)]
    return cells


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_sampled_parity_and_conservation_8192(oracle, storage):
    require_gpu()
    rng = np.random.default_rng(40)
    rg, rl = W.unit_cs_coexistence(0.8)
    rho0 = W.smooth_random(N, N, 41, mean=0.5 * (rg + rl), amplitude=0.45 * (rl - rg), modes=6)
    rho0 += W.noise((N, N), 42)
    p = W.params(N, N, tr=0.8, storage=storage)
    p["rho_ref"] = W.shift_reference(rho0, storage)
    lat = gpu_lattice(p, rho0)
    launch = lat.launch()
    log(f"case {storage} {N}x{N}, launch {launch}")
    d0 = lat.diagnostics()
    lat.step(5)
    cells = _samples(launch, rng)
    f = lat.populations()
    idx = np.arange(-2, 3)
    patches = []
    for x, y in cells:
        ys = torch.as_tensor((y + idx) % N, device=f.device)
        xs = torch.as_tensor((x + idx) % N, device=f.device)
        patches.append(f[:, ys][:, :, xs].cpu().numpy())
    del f
    lat.step(1)
    f1 = lat.populations()
    got = [f1[:, y, x].cpu().numpy() for x, y in cells]
    del f1
    q = dict(p)
    q["nx"] = q["ny"] = 5
    P5 = oracle_params(oracle, q)
    worst = 0.0
    for (x, y), patch, g in zip(cells, patches, got):
        h = np.ascontiguousarray(patch)
        oracle.step(P5, h, 1)
        err = np.abs(g - h[:, 2, 2]).max() / np.abs(h[:, 2, 2]).max()
        worst = max(worst, err)
        assert err <= TOL[storage], (x, y, err)
    d1 = lat.diagnostics()
    lat.sync()
    dm = abs(d1["mass"] / d0["mass"] - 1)
    mom = max(abs(d1["mom_x"]), abs(d1["mom_y"])) / (d0["mass"] * CS)
    log(f"  {len(cells)} sampled cells, worst {worst:.2e}; mass {dm:.1e}, momentum {mom:.1e}")
    assert dm < (1e-12 if storage == "f64" else 1e-5)
    assert mom < (1e-12 if storage == "f64" else 1e-5)

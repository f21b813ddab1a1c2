"""The two-step pass (two time steps per launch; the first step's result stays
on chip, rounded to the storage type) through the C ABI.

It computes each step with the same device routines as a single step, on a
tile widened by three columns and three rows on each side, so its populations
must equal those of single steps bit for bit, in every storage mode (the
per-cell FP16 mode hands its new reference densities over too), with either
collision, in every launch shape, on ragged and tiny lattices,
from even or odd starting times, and the first domain error it reports must
be the oracle's (same step, same cell) whichever step of a pair it falls in.
Beside that, parity with the FP64 oracle directly (the tolerance of the other
parity tests)."""
import numpy as np
import pytest
import torch

from paper_2003_07968_amd import workloads as W

from .gpu_common import assert_parity, gpu_lattice, gpu_state, log, oracle_state, require_gpu
from .helpers import oracle_params

pytestmark = pytest.mark.gpu

# (block_x, seg_rows) of the two-step pass: several strips and segments, one
# row per segment, one segment for the whole lattice
SHAPES = [(128, 1), (256, 5), (256, 16), (512, 203)]


def _smooth_case(nx, ny, storage="f64", collision="bgk", seed=12):
    p = W.params(nx, ny, tr=0.8, storage=storage, collision=collision)
    rg, rl = W.unit_cs_coexistence(0.8)
    rho0 = W.smooth_random(nx, ny, seed, mean=0.5 * (rg + rl), amplitude=0.5 * (rl - rg))
    p["rho_ref"] = W.shift_reference(rho0, storage)
    return p, rho0


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "f16l"])
def test_two_step_pass_bitwise_equals_single_steps(storage, collision):
    require_gpu()
    p, rho0 = _smooth_case(301, 203, storage, collision)
    ref = gpu_lattice(p, rho0, launch=(256, 8))
    assert ref.fusion() == 1
    ref.step(25)
    f_ref = ref.populations()
    for shape in SHAPES:
        lat = gpu_lattice(p, rho0, fusion=(2,) + shape)
        assert lat.fusion() == 2 and lat.launch()[:2] == shape
        lat.step(25)  # twelve passes, then one single step
        lat.sync()
        assert torch.equal(lat.populations(), f_ref), shape


def test_pairs_from_an_odd_time():
    require_gpu()
    p, rho0 = _smooth_case(160, 96, "f64", "mrt", seed=13)
    ref = gpu_lattice(p, rho0, launch=(128, 7))
    ref.step(17)
    lat = gpu_lattice(p, rho0, fusion=(2, 256, 7))
    for n in (1, 4, 3, 9):   # passes start at t = 1, 3, 5, then 8, 10, 12, 14
        lat.step(n)
    from paper_2003_07968_amd import lbm
    assert lbm.lbm_time(lat.handle) == 17
    assert torch.equal(lat.populations(), ref.populations())


@pytest.mark.parametrize("storage", ["f64", "f16l"])
@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4), (17, 9), (250, 7), (251, 31)])
def test_tiny_and_ragged_lattices(nx, ny, storage):
    # lattices narrower than the halo (columns and rows wrap several times
    # within one tile) and widths at and past one strip of 256 threads; the
    # per-cell mode also exchanges its reference densities between lanes
    require_gpu()
    p, rho0 = _smooth_case(nx, ny, storage, "bgk", seed=14)
    ref = gpu_lattice(p, rho0, launch=(64, 1))
    ref.step(10)
    for shape in ((128, 1), (256, 3), (256, ny)):
        lat = gpu_lattice(p, rho0, fusion=(2,) + shape)
        lat.step(10)
        lat.sync()
        assert torch.equal(lat.populations(), ref.populations()), (nx, ny, storage, shape)


def test_fp64_two_step_pass_matches_oracle(oracle):
    require_gpu()
    p, rho0 = W.droplet_64(seed=3)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0, fusion=(2, 128, 5))
    for target, t in ((2, 0), (30, 2), (100, 30)):
        lat.step(target - t)
        oracle.step(P, f, target - t)
        assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what=f"t={target}")
    lat.sync()


def test_defaults_and_rejected_arguments():
    require_gpu()
    from paper_2003_07968_amd import lbm
    # default shape on a small lattice: one strip, segments of the minimum
    # length, 2 rows (more workgroups beat the halo rows when the lattice
    # cannot fill the device)
    for storage in ("f64", "f32", "f16", "f16l"):
        p, rho0 = _smooth_case(64, 48, storage)
        lat = gpu_lattice(p, rho0)
        assert lat.fusion() == 2
        assert lat.launch() == (256, 2, 24), storage
    p, rho0 = _smooth_case(64, 48)
    lat = gpu_lattice(p, rho0)
    for bad in ((3,), (0,), (2, 192), (2, 64), (2, 256, -1)):
        with pytest.raises(lbm.LbmError) as e:
            lat.set_fusion(*bad)
        assert e.value.status == lbm.LBM_ERR_INVALID_ARG, bad
    assert lat.fusion() == 2 and lat.launch()[:2] == (256, 2)
    lat.set_fusion(1)
    assert lat.fusion() == 1


def _converging_disk(rho_disk, speed, nx=24, ny=20, cx=7, cy=13):
    """A disk of radius 3 at rho_disk in a rho = 0.2 gas, moving radially inward
    at `speed`: at T_r = 0.8 (EOS domain rho < ~0.47) the centre leaves the
    domain at step 1 (the oracle's step 0 is clean)."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    dx, dy = xx - cx, yy - cy
    r = np.hypot(dx, dy)
    rho0 = np.full((ny, nx), 0.2)
    rho0[r <= 3] = rho_disk
    ring = (r <= 3) & (r > 0)
    ux = np.where(ring, -speed * dx / np.maximum(r, 1), 0.0)
    uy = np.where(ring, -speed * dy / np.maximum(r, 1), 0.0)
    return rho0, ux, uy


@pytest.mark.parametrize("lead", [0, 1])
@pytest.mark.parametrize("disk", [(0.45, 0.05), (0.40, 0.09), (0.46, 0.10)])
def test_domain_error_same_step_and_cell(oracle, disk, lead):
    # lead = 0: the first failing step (1) is the second step of the first
    # pass; lead = 1 (one single step first): it is the first step of a pass
    require_gpu()
    from paper_2003_07968_amd import lbm
    rho0, ux, uy = _converging_disk(*disk)
    p = W.params(24, 20, tr=0.8)
    P = oracle_params(oracle, p)
    with pytest.raises(oracle.OracleError) as ref:
        oracle.step(P, oracle.init(P, rho0, ux, uy), 4)
    assert ref.value.fault.step == 1
    msgs = []
    for fusion in ((2, 128, 3), (2, 256, 20), (1,)):
        lat = gpu_lattice(p, rho0, ux, uy, fusion=fusion)
        lat.step(lead)
        lat.step(4 - lead)
        with pytest.raises(lbm.LbmError) as e:
            lat.sync()
        assert e.value.status == lbm.LBM_ERR_DOMAIN
        msgs.append(lbm.lbm_last_error(lat.handle))
    log(f"  {msgs[0]}")
    assert len(set(msgs)) == 1, msgs
    assert (f"step {ref.value.fault.step}," in msgs[0]
            and f"cell {ref.value.fault.cell} " in msgs[0])


def test_random_sizes_and_shapes_bitwise():
    # seeded draws of lattice sizes around strip and segment boundaries,
    # launch shapes, storage modes and collisions: the two-step pass equals
    # single steps bit for bit in every draw
    require_gpu()
    rng = np.random.default_rng(21)
    storages = ["f64", "f32", "f16", "f16l"]
    for k in range(12):
        bx = int(rng.choice([128, 256, 512]))
        width = (bx - 6) // 32 * 32
        nx = int(max(3, width * int(rng.integers(1, 4)) + int(rng.integers(-3, 4))))
        ny = int(rng.integers(3, 90))
        rows = int(rng.integers(1, ny + 1))
        storage = storages[k % 4]
        collision = "mrt" if k % 3 == 0 else "bgk"
        p, rho0 = _smooth_case(nx, ny, storage, collision, seed=100 + k)
        steps = int(rng.integers(2, 9))
        ref = gpu_lattice(p, rho0, launch=(64, 3))
        ref.step(steps)
        lat = gpu_lattice(p, rho0, fusion=(2, bx, rows))
        lat.step(steps)
        lat.sync()
        case = (nx, ny, bx, rows, storage, collision, steps)
        log(f"  case {case}")
        assert torch.equal(lat.populations(), ref.populations()), case

"""HIP path (through the C ABI) against the CPU oracle on the same seeded
inputs: element-by-element, per field, normwise within PARITY_TOL.

Sizes span one to many workgroup tiles, ragged strips and row segments,
non-square lattices and the 3-cell minimum; the 64 x 64 droplet runs the
full 5000 steps; the 2048 x 2048 slabs are compared over their first steps
at full size, alone and as the benchmark runs them (the four lattices in
one batched launch, in the benchmark's launch shape)."""
import numpy as np
import pytest
import torch

from paper_2003_07968_amd import workloads as W

from .gpu_common import (assert_parity, gpu_lattice, gpu_state, log, oracle_state,
                         require_gpu)
from .helpers import oracle_params

pytestmark = pytest.mark.gpu


def _smooth_case(nx, ny, seed, tr=0.8, **kw):
    p = W.params(nx, ny, tr=tr, **kw)
    rg, rl = W.unit_cs_coexistence(tr)
    rho0 = W.smooth_random(nx, ny, seed, mean=0.5 * (rg + rl), amplitude=0.5 * (rl - rg))
    return p, rho0


@pytest.mark.parametrize("nx,ny", [(3, 3), (13, 11), (64, 64), (130, 67), (300, 257),
                                   (517, 5)])
def test_one_and_ten_steps_match_oracle(oracle, nx, ny):
    require_gpu()
    log(f"case one/ten steps nx={nx} ny={ny}")
    p, rho0 = _smooth_case(nx, ny, seed=nx * 1000 + ny)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what="t=0")
    lat.step(1)
    oracle.step(P, f, 1)
    assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what="t=1")
    lat.step(9)
    oracle.step(P, f, 9)
    assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what="t=10")
    lat.sync()


def test_droplet_64_full_run(oracle):
    # 64 x 64 droplet, R0 = 16, W = 2, T_r = 0.8, tau = 1, seeded noise:
    # the oracle's reference case, compared at t = 1, 10, 100, 1000, 5000.
    require_gpu()
    log("case droplet 64x64, 5000 steps")
    p, rho0 = W.droplet_64(seed=1)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    t = 0
    for target in (1, 10, 100, 1000, 5000):
        lat.step(target - t)
        oracle.step(P, f, target - t)
        t = target
        assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what=f"t={t}")
    lat.sync()
    assert lat.t == 5000


@pytest.mark.parametrize("variant", [
    {"force_on": False, "tau": 0.7},
    {"m2_trace_alt": True, "sigma": 2.5},
    {"epsilon": 0.0, "sigma": 1.0},
    {"sigma": 0.125, "tau": 0.6},
    {"G": -3.0},
])
def test_parameter_variants(oracle, variant):
    require_gpu()
    log(f"case variant {variant}")
    kw = dict(variant)
    G = kw.pop("G", None)
    p, rho0 = _smooth_case(40, 36, seed=5, **kw)
    if G is not None:
        p["G"] = G
    P = oracle_params(oracle, p)
    rng = np.random.default_rng(5)
    ux0 = rng.uniform(-0.02, 0.02, rho0.shape)
    uy0 = rng.uniform(-0.02, 0.02, rho0.shape)
    f = oracle.init(P, rho0, ux0, uy0)
    lat = gpu_lattice(p, rho0, ux0, uy0)
    lat.step(50)
    oracle.step(P, f, 50)
    assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what="t=50")


def test_paper_eos_droplet(oracle):
    # The paper's own EOS set (Sec. IV.A), W = 5, tau = 0.8, sigma = 0.5.
    require_gpu()
    log("case paper EOS droplet 80x72")
    p = W.params(80, 72, tr=0.8, eos="paper", tau=0.8, sigma=0.5)
    rho0 = W.droplet(80, 72, 20.0, 2.3550, 0.1665, 5.0) + W.noise((72, 80), 11)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    lat.step(500)
    oracle.step(P, f, 500)
    assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what="t=500")


def test_full_size_slab_first_steps(oracle):
    # 2048 x 2048 slab at T_r = 0.7 stepped alone (the library's default: one
    # two-step launch in the default shape), compared element by element at
    # t = 2; then one single-step launch (an odd remainder), compared at t = 3.
    require_gpu()
    log("case slab 2048x2048, 2 + 1 steps")
    p, rho0 = W.slab_case(n=2048, tr=0.7)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    assert lat.fusion() == 2
    log(f"  launch {lat.launch()}")
    for n, t in ((2, 2), (1, 3)):
        lat.step(n)
        oracle.step(P, f, n)
        assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what=f"t={t}")


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_full_size_batch_as_benchmarked(oracle, collision):
    # the benchmark's own form: the four 2048 x 2048 slabs (T_r 0.6 .. 0.9)
    # in one batch, one launch for all four per two steps, in the launch
    # shape bench.py uses (BGK, the default line, and MRT, --collision mrt);
    # every lattice compared element by element with the oracle at t = 2 (one
    # two-step launch) and t = 3 (one single step)
    require_gpu()
    import bench
    from paper_2003_07968_amd import lbm
    shape = bench.SLAB_LAUNCH[2]["f64"]
    log(f"case four 2048x2048 slabs as one batch, {collision}, launch {shape}, 2 + 1 steps")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cases = [W.slab_case(n=bench.N, tr=tr) for tr in bench.TEMPS]
        for p, _ in cases:
            p["collision"] = W.COLLISION[collision]
        lats = [gpu_lattice(p, rho0) for p, rho0 in cases]
        batch = lbm.Batch(len(lats))
        for lat in lats:
            batch.add(lat)
        batch.set_launch(2, *shape)
        assert batch.launch() == (2,) + tuple(shape)
        refs = []
        for p, rho0 in cases:
            P = oracle_params(oracle, p)
            refs.append((P, oracle.init(P, rho0)))
        for n, t in ((2, 2), (1, 3)):
            batch.step(n)
            torch.cuda.synchronize()
            for lat, (P, f), tr in zip(lats, refs, bench.TEMPS):
                oracle.step(P, f, n)
                assert lat.t == t
                assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what=f"T_r={tr} t={t}")
        for lat in lats:
            lat.sync()


def test_full_size_batch_graph_replays(oracle):
    # the benchmarked form over 96 steps: twelve replays of the batch's
    # captured eight-step graph (four two-step launches each) at full size,
    # every lattice compared with the oracle at the end
    require_gpu()
    import bench
    from paper_2003_07968_amd import lbm
    shape = bench.SLAB_LAUNCH[2]["f64"]
    log(f"case four 2048x2048 slabs as one batch, launch {shape}, 96 steps in graphs")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cases = [W.slab_case(n=bench.N, tr=tr) for tr in bench.TEMPS]
        lats = [gpu_lattice(p, rho0) for p, rho0 in cases]
        batch = lbm.Batch(len(lats))
        for lat in lats:
            batch.add(lat)
        batch.set_launch(2, *shape)
        batch.step(96)
        torch.cuda.synchronize()
        for lat, (p, rho0), tr in zip(lats, cases, bench.TEMPS):
            P = oracle_params(oracle, p)
            f = oracle.init(P, rho0)
            oracle.step(P, f, 96)
            assert lat.t == 96
            assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what=f"T_r={tr} t=96")
        for lat in lats:
            lat.sync()


@pytest.mark.parametrize("tr", [0.6, 0.7, 0.8, 0.9])
def test_full_size_slab_conservation(tr):
    # 2048 x 2048 slab: mass and total momentum are conserved to rounding over
    # 500 steps (properties that hold at any size).
    require_gpu()
    log(f"case slab 2048x2048 T_r={tr} conservation")
    p, rho0 = W.slab_case(n=2048, tr=tr)
    lat = gpu_lattice(p, rho0)
    d0 = lat.diagnostics()
    lat.step(500)
    d1 = lat.diagnostics()
    lat.sync()
    assert abs(d1["mass"] / d0["mass"] - 1) < 1e-12
    scale = d0["mass"] * (1 / 3) ** 0.5
    assert abs(d1["mom_x"] - d0["mom_x"]) < 1e-12 * scale
    assert abs(d1["mom_y"] - d0["mom_y"]) < 1e-12 * scale
    assert np.isfinite(d1["umax"]) and d1["umax"] < 0.3


@pytest.mark.parametrize("launch", [(64, 1), (64, 7), (128, 3), (192, 64), (256, 5), (512, 2),
                                    (320, 1000)])
def test_launch_shapes_bitwise_identical(launch):
    # Every tile shape must give the same bits: a race or a missing barrier in
    # the LDS exchange would show up here.
    require_gpu()
    log(f"case launch shape {launch}")
    p, rho0 = _smooth_case(301, 203, seed=12)
    ref = gpu_lattice(p, rho0)
    ref.step(20)
    lat = gpu_lattice(p, rho0, launch=launch)
    lat.step(20)
    assert torch.equal(ref.populations(), lat.populations())
    a, b = ref.moments(), lat.moments()
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_repeat_runs_bitwise_identical():
    require_gpu()
    p, rho0 = W.droplet_64(seed=3)
    a = gpu_lattice(p, rho0)
    b = gpu_lattice(p, rho0)
    a.step(200)
    b.step(200)
    assert torch.equal(a.populations(), b.populations())
    assert a.diagnostics() == b.diagnostics()


def test_checkpoint_restart_bitwise():
    require_gpu()
    p, rho0 = W.droplet_64(seed=4)
    a = gpu_lattice(p, rho0)
    a.step(80)
    b = gpu_lattice(p, rho0)
    b.step(37)
    f = b.populations()
    c = gpu_lattice(p, rho0)
    c.set_populations(f, 37)
    c.step(43)
    assert c.t == 80
    assert torch.equal(a.populations(), c.populations())


def test_set_get_populations_roundtrip(oracle):
    require_gpu()
    p, rho0 = _smooth_case(21, 17, seed=8)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    oracle.step(P, f, 3)
    lat = gpu_lattice(p, rho0)
    lat.set_populations(torch.from_numpy(f).cuda(), 3)
    assert np.array_equal(lat.populations().cpu().numpy(), f)
    lat.step(4)
    oracle.step(P, f, 4)
    assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what="after restart")


def test_diagnostics_match_oracle(oracle):
    require_gpu()
    p, rho0 = W.droplet_64(seed=1)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    rho_prev = oracle.moments(P, f)["rho"]
    lat.step(100)
    oracle.step(P, f, 100)
    g = lat.diagnostics()
    o = oracle.diagnostics(P, f, rho_prev)
    log(f"  gpu {g}\n  cpu {o}")
    assert abs(g["mass"] - o["mass"]) <= 1e-13 * o["mass"]
    scale = o["mass"] * (1 / 3) ** 0.5
    assert abs(g["mom_x"] - o["mom_x"]) <= 1e-12 * scale
    assert abs(g["mom_y"] - o["mom_y"]) <= 1e-12 * scale
    assert abs(g["ssc_num"] - o["ssc_num"]) <= 1e-10 * o["ssc_num"]
    assert abs(g["ssc_den"] - o["ssc_den"]) <= 1e-13 * o["ssc_den"]
    assert abs(g["umax"] - o["umax"]) <= 1e-10 * o["umax"]
    # the snapshot moved to t = 100: a second call without steps gives 0
    assert lat.diagnostics()["ssc_num"] == 0.0


def test_domain_error_matches_oracle(oracle):
    require_gpu()
    from paper_2003_07968_amd import lbm
    nx, ny = 24, 20
    p = W.params(nx, ny, tr=0.8)
    rho0 = np.full((ny, nx), 0.2)
    rho0[13, 7] = 0.95   # psi^2 < 0 above the EOS's rho_max
    rho0[15, 2] = 0.97
    P = oracle_params(oracle, p)
    with pytest.raises(oracle.OracleError) as ref:
        oracle.step(P, oracle.init(P, rho0), 3)
    lat = gpu_lattice(p, rho0)
    lat.step(3)
    with pytest.raises(lbm.LbmError) as e:
        lat.sync()
    assert e.value.status == lbm.LBM_ERR_DOMAIN
    msg = lbm.lbm_last_error(lat.handle)
    log(f"  {msg}")
    assert f"step {ref.value.fault.step}," in msg and f"cell {ref.value.fault.cell} " in msg
    # sticky: later calls report it again
    with pytest.raises(lbm.LbmError):
        lat.moments()


def test_invalid_arguments_rejected():
    require_gpu()
    from paper_2003_07968_amd import lbm
    p, rho0 = W.droplet_64()
    for bad in ({"tau": 0.5}, {"G": 0.0}, {"nx": 2}, {"storage": 7}):
        q = dict(p)
        q.update(bad)
        if "nx" in bad:
            r = rho0[:, :2]
        else:
            r = rho0
        with pytest.raises(lbm.LbmError) as e:
            lbm.Lattice(q, r)
        assert e.value.status == lbm.LBM_ERR_INVALID_ARG
    lat = gpu_lattice(p, rho0)
    with pytest.raises(lbm.LbmError):
        lat.step(-1)
    with pytest.raises(lbm.LbmError):
        lat.set_launch(100, 4)
    assert lat.t == 0

"""The MRT collision (Eqs. MRTCO, GFSMRT, Appendix A) on the GPU through the
C ABI, against the CPU oracle: FP64 parity per field at the 1e-12 bar, the
paper's droplet-oscillation setup of Sec. IV.C, equal rates against the
BGK kernel, the reduced-precision storage modes against the
storage-emulating oracle, and batches bitwise equal to lattices run alone."""
import numpy as np
import pytest
import torch

from oracle import analytics as A
from paper_2003_07968_amd import lbm
from paper_2003_07968_amd import workloads as W

from .gpu_common import assert_parity, gpu_lattice, gpu_state, log, oracle_state, require_gpu
from .helpers import fit_damped_period, oracle_params, x_extent
from .test_gpu_storage import EMULATED_TOL

pytestmark = pytest.mark.gpu

RATES = [(1.0, 1.0, 1.0, 1.0, 1.0), (1.7, 0.8, 1.3, 0.6, 1.1)]


def _field(nx, ny, seed, tr=0.8):
    rg, rl = W.unit_cs_coexistence(tr)
    return W.smooth_random(nx, ny, seed, mean=0.5 * (rg + rl), amplitude=0.45 * (rl - rg))


@pytest.mark.parametrize("nx,ny", [(3, 3), (13, 11), (64, 64), (130, 67), (517, 5)])
@pytest.mark.parametrize("rates", RATES)
def test_mrt_steps_match_oracle(oracle, nx, ny, rates):
    require_gpu()
    p = W.params(nx, ny, tr=0.8, tau=0.65, collision="mrt", mrt=rates)
    rho0 = _field(nx, ny, 31)
    log(f"case mrt {nx}x{ny} rates={rates}")
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    for target, t in ((1, 0), (10, 1), (60, 10)):
        lat.step(target - t)
        oracle.step(P, f, target - t)
        assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what=f"t={target}")
    lat.sync()


def _paper_ellipse(tr):
    n = 200
    rg, rl = A.maxwell(A.PAPER_EOS, tr)[:2]
    p = W.params(n, n, tr=tr, tau=0.65, eos="paper", collision="mrt")
    return p, W.ellipse(n, n, 30.0, 27.0, rl, rg, 5.0), 0.5 * (rg + rl)


def test_paper_oscillation_parity_and_period(oracle):
    # Sec. IV.C at T_r = 0.6: element-wise parity after 400 steps, then the
    # period over 4000 steps against the printed T_n = 3200 (3 %, the paper's
    # 100-step sampling) and against the oracle's own period (FP64 parity
    # makes the two time series agree to rounding).
    require_gpu()
    p, rho0, rho_m = _paper_ellipse(0.6)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    ts, rs_g, rs_o = [], [], []
    rho = torch.empty((200, 200), dtype=torch.float64, device="cuda")
    for k in range(201):
        if k:
            lat.step(20)
            oracle.step(P, f, 20)
        if k == 20:
            assert_parity(gpu_state(lat), oracle_state(oracle, P, f), what="t=400")
        lbm.lbm_moments(lat.handle, rho=rho)
        ts.append(20 * k)
        rs_g.append(x_extent(rho[99:101].cpu().numpy(), rho_m))
        rs_o.append(x_extent(oracle.moments(P, f)["rho"][99:101], rho_m))
    lat.sync()
    Tg = fit_damped_period(ts, rs_g)[0]
    To = fit_damped_period(ts, rs_o)[0]
    log(f"  period gpu {Tg:.1f}, oracle {To:.1f}, paper 3200; extent max diff "
        f"{np.abs(np.array(rs_g) - np.array(rs_o)).max():.2e}")
    assert np.abs(np.array(rs_g) - np.array(rs_o)).max() < 1e-8
    assert abs(Tg / To - 1) < 1e-6
    assert abs(Tg / 3200.0 - 1) < 0.03


def test_equal_rates_give_the_bgk_result():
    require_gpu()
    n, tau = 96, 0.7
    rg, rl = W.unit_cs_coexistence(0.8)
    rho0 = W.droplet(n, n, 24.0, rl, rg, 2.0) + W.noise((n, n), 4)
    a = gpu_lattice(W.params(n, n, tau=tau), rho0)
    b = gpu_lattice(W.params(n, n, tau=tau, collision="mrt", mrt=(tau,) * 5), rho0)
    a.step(300)
    b.step(300)
    fa, fb = a.populations(), b.populations()
    assert float((fa - fb).abs().max() / fa.abs().max()) < 1e-13


@pytest.mark.parametrize("storage", ["f32", "f16", "f16l"])
def test_mrt_reduced_storage_matches_emulating_oracle(oracle, storage):
    require_gpu()
    p, rho0 = W.droplet_64(seed=1)
    p.update(W.params(64, 64, tr=0.8, tau=0.65, collision="mrt", mrt=RATES[1]))
    p["storage"] = W.STORAGE[storage]
    p["rho_ref"] = W.shift_reference(rho0, storage)
    P = oracle_params(oracle, p)
    f = oracle.init(P, rho0)
    lat = gpu_lattice(p, rho0)
    lat.step(100)
    oracle.step(P, f, 100)
    from .gpu_common import parity_errors
    errs = parity_errors(gpu_state(lat), oracle_state(oracle, P, f))
    log(f"  mrt {storage}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for v in errs.values():
        assert v <= EMULATED_TOL[storage]
    lat.sync()


@pytest.mark.parametrize("launch", [(64, 1), (128, 7), (256, 8), (512, 3)])
def test_mrt_launch_shapes_bitwise_identical(launch):
    require_gpu()
    p = W.params(301, 203, tr=0.8, tau=0.65, collision="mrt", mrt=RATES[1])
    rho0 = _field(301, 203, 12)
    ref = gpu_lattice(p, rho0)
    ref.step(20)
    lat = gpu_lattice(p, rho0, launch=launch)
    lat.step(20)
    assert torch.equal(ref.populations(), lat.populations())


def test_mrt_batch_equals_alone():
    require_gpu()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cases = []
        for k, side in enumerate((40, 72, 130)):
            p = W.params(side, side - 7, tr=0.75, tau=0.65, collision="mrt", mrt=RATES[k % 2])
            cases.append((p, _field(side, side - 7, 50 + k, tr=0.75)))
        solo = [gpu_lattice(p, r) for p, r in cases]
        mates = [gpu_lattice(p, r) for p, r in cases]
        batch = lbm.Batch(len(cases))
        for m in mates:
            batch.add(m)
        # a BGK lattice does not join an MRT batch
        with pytest.raises(lbm.LbmError):
            batch.add(gpu_lattice(W.params(40, 40, tr=0.75), _field(40, 40, 1, tr=0.75)))
        batch.step(19)
        for x in solo:
            x.step(19)
        for x, m in zip(solo, mates):
            assert torch.equal(x.populations(), m.populations())
    torch.cuda.synchronize()


def test_mrt_invalid_rates_rejected():
    require_gpu()
    p = W.params(16, 16, tau=0.65, collision="mrt", mrt=(1.0, 0.5, 1.0, 1.0, 1.0))
    with pytest.raises(lbm.LbmError):
        gpu_lattice(p, _field(16, 16, 2))
    q = W.params(16, 16, tau=0.65)
    q["collision"] = 7
    with pytest.raises(lbm.LbmError):
        gpu_lattice(q, _field(16, 16, 2))

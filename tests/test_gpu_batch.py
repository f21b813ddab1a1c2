"""Batched stepping (one kernel launch per two steps, or per step, for many
lattices, HIP graph replays) and the autotuner, through the C ABI.  A batched
lattice must give exactly the bits it gives when stepped alone."""
import numpy as np
import pytest
import torch

from paper_2003_07968_amd import lbm
from paper_2003_07968_amd import workloads as W

from .gpu_common import (PARITY_TOL, assert_parity, gpu_lattice, gpu_state, log,
                         oracle_state, require_gpu)
from .helpers import oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def side_stream():
    # batches capture HIP graphs, which the legacy null stream does not allow;
    # run every test on a stream of its own (default priority)
    require_gpu()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        yield s
    torch.cuda.synchronize()


def _mixed(storage="f64", count=6, seed=3):
    return W.batch_case(count=count, seed=seed, storage=storage, side_range=(24, 160))


@pytest.mark.parametrize("fusion", [2, 1])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "f16l"])
def test_batch_equals_alone(storage, fusion):
    # eager launches (3 steps: one two-step launch and a single step), then
    # graph replays (8-step graphs) with checks and eager work in between,
    # one single step that flips the launch parity, then remainders: every
    # lattice bitwise equal to its solo run after each stage.
    require_gpu()
    cases = _mixed(storage)
    solo = [gpu_lattice(p, r) for p, r in cases]
    mates = [gpu_lattice(p, r) for p, r in cases]
    batch = lbm.Batch(len(cases))
    batch.set_fusion(fusion)
    for lat in mates:
        batch.add(lat)
    assert batch.fusion() == fusion
    done = 0
    for n in (3, 8, 8, 1, 16, 5, 2):
        batch.step(n)
        for s in solo:
            s.step(n)
        done += n
        _ = torch.zeros(4, device="cuda").sum().item()  # unrelated eager work
        for k, (s, m) in enumerate(zip(solo, mates)):
            assert m.t == s.t == done
            assert torch.equal(s.populations(), m.populations()), (storage, k, done)
    for m in mates:
        m.sync()


def test_membership_changes_and_outside_steps():
    require_gpu()
    cases = _mixed("f64", count=5, seed=4)
    solo = [gpu_lattice(p, r) for p, r in cases]
    mates = [gpu_lattice(p, r) for p, r in cases]
    batch = lbm.Batch(8)
    for lat in mates[:3]:
        batch.add(lat)
    batch.step(9)
    for s in solo[:3]:
        s.step(9)
    # a lattice joins late, one leaves, one is stepped on its own
    batch.add(mates[3])
    batch.remove(mates[0])
    mates[1].step(2)
    solo[1].step(2)
    batch.step(11)
    for k in (1, 2, 3):
        solo[k].step(11)
    assert len(batch) == 3
    for k in range(4):
        assert mates[k].t == solo[k].t
        assert torch.equal(solo[k].populations(), mates[k].populations()), k
    with pytest.raises(lbm.LbmError):
        batch.add(mates[1])  # already a member


def test_batch_fusion_switch_midway_and_bad_argument():
    require_gpu()
    cases = _mixed("f32", count=3, seed=10)
    solo = [gpu_lattice(p, r) for p, r in cases]
    mates = [gpu_lattice(p, r) for p, r in cases]
    batch = lbm.Batch(3)
    for m in mates:
        batch.add(m)
    assert batch.fusion() == 2
    batch.step(9)
    batch.set_fusion(1)
    batch.step(10)
    batch.set_fusion(2)
    batch.step(13)
    for s in solo:
        s.step(32)
    for s, m in zip(solo, mates):
        assert m.t == 32 and torch.equal(s.populations(), m.populations())
    for bad in (0, 3, -1):
        with pytest.raises(lbm.LbmError):
            batch.set_fusion(bad)
    assert batch.fusion() == 2


@pytest.mark.parametrize("storage", ["f64", "f16l"])
def test_batch_set_launch_shapes_and_bad_arguments(storage):
    # explicit launch shapes, two-step and single-step, switched between
    # calls (graph replays included): every lattice bitwise equal to its solo
    # run; bad shapes are rejected and leave the launch as it was
    require_gpu()
    cases = _mixed(storage, count=4, seed=12)
    solo = [gpu_lattice(p, r) for p, r in cases]
    mates = [gpu_lattice(p, r) for p, r in cases]
    batch = lbm.Batch(4)
    for m in mates:
        batch.add(m)
    done = 0
    for steps, bx, rows, n in ((2, 256, 37, 17), (2, 128, 3, 10), (1, 64, 3, 9),
                               (2, 512, 0, 16), (1, 320, 17, 5), (2, 256, 1, 11)):
        batch.set_launch(steps, bx, rows)
        got = batch.launch()
        assert got[:2] == (steps, bx) and (rows == 0 or got[2] == rows), got
        batch.step(n)
        done += n
        for s in solo:
            s.step(n)
        for s, m in zip(solo, mates):
            assert m.t == done and torch.equal(s.populations(), m.populations()), (steps, bx, rows)
    before = batch.launch()
    for bad in ((3, 256, 8), (0, 256, 8), (2, 192, 8), (2, 256, -1), (1, 96, 4), (1, 576, 4),
                (1, 256, 0)):
        with pytest.raises(lbm.LbmError):
            batch.set_launch(*bad)
        assert batch.launch() == before, bad


def test_batch_rejects_mixed_storage_and_full():
    require_gpu()
    (p1, r1), (p2, r2) = _mixed("f64", count=2, seed=5)
    a = gpu_lattice(p1, r1)
    p2 = dict(p2)
    p2["storage"], p2["rho_ref"] = 1, float(r2.mean())
    b = gpu_lattice(p2, r2)
    batch = lbm.Batch(1)
    batch.add(a)
    with pytest.raises(lbm.LbmError):
        batch.add(b)
    batch2 = lbm.Batch(1)
    batch2.add(b)
    with pytest.raises(lbm.LbmError):
        batch2.add(a)


def test_autotune_keeps_state():
    require_gpu()
    p, rho0 = W.slab_case(n=512, ny=384, tr=0.8)
    lat = gpu_lattice(p, rho0)
    lat.step(7)
    before = lat.populations().clone()
    bx, rows, us = lat.autotune()
    log(f"  autotune 512x384: block {bx}, rows {rows}, {us:.1f} us/step")
    assert lat.t == 7 and torch.equal(before, lat.populations())
    assert lat.launch()[:2] == (bx, rows)
    ref = gpu_lattice(p, rho0)
    ref.step(10)
    lat.step(3)
    assert torch.equal(ref.populations(), lat.populations())


def test_batch_autotune_keeps_state():
    require_gpu()
    cases = _mixed("f32", count=4, seed=7)
    mates = [gpu_lattice(p, r) for p, r in cases]
    batch = lbm.Batch(4)
    for m in mates:
        batch.add(m)
    batch.step(5)
    before = [m.populations().clone() for m in mates]
    bx, rows, us = batch.autotune()
    log(f"  batch autotune: block {bx}, rows {rows}, {us:.1f} us/step")
    for m, b0 in zip(mates, before):
        assert m.t == 5 and torch.equal(b0, m.populations())
    solo = [gpu_lattice(p, r) for p, r in cases]
    for s in solo:
        s.step(12)
    batch.step(7)
    for s, m in zip(solo, mates):
        assert torch.equal(s.populations(), m.populations())


def test_domain_error_stays_with_its_lattice():
    require_gpu()
    cases = _mixed("f64", count=3, seed=8)
    p, r = cases[1]
    r = r.copy()
    r[2, 3] = 0.95  # above the EOS's rho_max: psi^2 < 0
    cases[1] = (p, r)
    mates = [gpu_lattice(p, rr) for p, rr in cases]
    batch = lbm.Batch(3)
    for m in mates:
        batch.add(m)
    batch.step(4)
    mates[0].sync()
    mates[2].sync()
    with pytest.raises(lbm.LbmError) as e:
        mates[1].sync()
    assert e.value.status == lbm.LBM_ERR_DOMAIN
    assert "step 0," in lbm.lbm_last_error(mates[1].handle)


def test_batch_on_null_stream_runs_eagerly():
    # on the legacy null stream no graph is captured; results are the same
    cases = _mixed("f64", count=2, seed=9)
    with torch.cuda.stream(torch.cuda.default_stream()):
        solo = [gpu_lattice(p, r) for p, r in cases]
        mates = [gpu_lattice(p, r) for p, r in cases]
        batch = lbm.Batch(2)
        for m in mates:
            batch.add(m)
        batch.step(19)
        for s in solo:
            s.step(19)
        for s, m in zip(solo, mates):
            assert torch.equal(s.populations(), m.populations())


@pytest.mark.parametrize("fusion", [2, 1])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_graph_replays_match_oracle(oracle, collision, fusion):
    # 40 batched FP64 steps: five replays of the captured 8-step graph, with
    # every lattice compared element by element with the CPU oracle after the
    # first replay and at the end (the graph path against the oracle, not
    # only against eager launches).
    require_gpu()
    cases = W.batch_case(count=3, seed=21, storage="f64", side_range=(20, 72))
    mates = []
    for p, r in cases:
        p = dict(p)
        if collision == "mrt":
            p.update(collision=W.COLLISION["mrt"], tau_e=0.9, tau_zeta=1.1, tau_q=1.2)
        mates.append((p, r, gpu_lattice(p, r)))
    batch = lbm.Batch(len(mates))
    batch.set_fusion(fusion)
    for _, _, lat in mates:
        batch.add(lat)
    fos = [(oracle_params(oracle, p), oracle.init(oracle_params(oracle, p), r))
           for p, r, _ in mates]
    done = 0
    for n in (8, 32):
        batch.step(n)
        done += n
        for (p, _, lat), (P, f) in zip(mates, fos):
            oracle.step(P, f, n)
            lat.sync()
            assert lat.t == done
            assert_parity(gpu_state(lat), oracle_state(oracle, P, f), PARITY_TOL,
                          f"{p['nx']}x{p['ny']} {collision} fusion {fusion} t={done}")

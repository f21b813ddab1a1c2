"""lbm_diagnostics_noalloc, the diagnostics entry point whose reduction scratch
is a static device array of the library, against lbm_diagnostics (whose
scratch is in the caller's workspace), through the C ABI: bitwise equal on
twin lattices, on two calls in a row, the second on a smaller lattice; a
sweep with more workgroups than the array holds is rejected before any
launch."""
import numpy as np
import pytest
import torch

from paper_2003_07968_amd import lbm
from paper_2003_07968_amd import workloads as W

from .gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu


def _twins(p, rho0, steps):
    a = lbm.Lattice(p, rho0)
    b = lbm.Lattice(p, rho0)
    a.step(steps)
    b.step(steps)
    return a, b


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_diagnostics_equal_workspace_diagnostics(storage):
    require_gpu()
    cases = [
        (W.slab_case(n=300, ny=257, tr=0.8), 11),            # many tiles, ragged strips
        ((W.params(64, 64, tr=0.8), W.droplet(64, 64, 16.0, *reversed(
            W.unit_cs_coexistence(0.8)), 2.0)), 7),          # smaller lattice second
    ]
    for (p, rho0), steps in cases:
        p = dict(p)
        p["storage"] = W.STORAGE[storage]
        p["rho_ref"] = W.shift_reference(rho0, storage)
        a, b = _twins(p, rho0, steps)
        for call in range(2):
            da = lbm.lbm_diagnostics(a.handle)
            db = lbm.lbm_diagnostics_noalloc(b.handle)
            log(f"  {p['nx']}x{p['ny']} {storage} call {call}: {db}")
            assert np.array_equal(np.array(da), np.array(db)), (da, db)
            a.step(3)
            b.step(3)
        # the steady-state snapshot was updated the same way by both
        assert lbm.lbm_diagnostics(a.handle) == lbm.lbm_diagnostics_noalloc(b.handle)


def test_noalloc_rejects_sweeps_beyond_the_static_scratch():
    require_gpu()
    p, rho0 = W.slab_case(n=1024, ny=1024, tr=0.8)
    lat = lbm.Lattice(p, rho0)
    lat.set_fusion(1)
    lat.set_launch(64, 1)          # 22 strips x 1024 one-row segments > 16384 workgroups
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_diagnostics_noalloc(lat.handle)
    assert ei.value.status == lbm.LBM_ERR_INVALID_ARG
    assert "16384" in str(ei.value)
    # the lattice is untouched and the workspace entry point still works
    d = lbm.lbm_diagnostics(lat.handle)
    assert np.isfinite(d).all()
    torch.cuda.synchronize()

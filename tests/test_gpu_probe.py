"""The bandwidth probe of the population access pattern (include/lbm_probe.h):
one pulled copy of nine FP64 planes, checked against its plain definition,
dst_i(x, y) = src_i(x - c_ix, y - c_iy) with periodic wrap, on sizes with
ragged strips and segments."""
import numpy as np
import pytest
import torch

from paper_2003_07968_amd import lbm

from .gpu_common import log, require_gpu

pytestmark = pytest.mark.gpu

# D2Q9 velocities in the library's population order
CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)


@pytest.mark.parametrize("nx,ny,rows", [(3, 3, 1), (37, 23, 5), (300, 41, 7), (513, 9, 32)])
def test_probe_is_a_pulled_copy(nx, ny, rows):
    require_gpu()
    log(f"case probe {nx}x{ny} rows {rows}")
    n = lbm.lbm_probe_stream_bytes(nx, ny) // 8
    plane = -(-nx // 16) * 16
    assert n == 9 * plane * ny
    rng = np.random.default_rng(nx * 1000 + ny)
    host = rng.standard_normal(n)
    src = torch.from_numpy(host).cuda()
    dst = torch.zeros_like(src)
    lbm.lbm_probe_stream(src, dst, nx, ny, rows)
    torch.cuda.synchronize()
    out = dst.cpu().numpy().reshape(ny, 9, plane)[:, :, :nx]
    f = host.reshape(ny, 9, plane)[:, :, :nx]
    for i in range(9):
        want = np.roll(np.roll(f[:, i, :], CY[i], axis=0), CX[i], axis=1)
        assert np.array_equal(out[:, i, :], want), i


def test_probe_rejects_bad_arguments():
    require_gpu()
    assert lbm.lbm_probe_stream_bytes(2, 10) == 0
    n = lbm.lbm_probe_stream_bytes(16, 16) // 8
    a = torch.zeros(n, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    for nx, ny, rows in ((2, 16, 4), (16, 2, 4), (16, 16, 0)):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_probe_stream(a, b, nx, ny, rows)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_probe_stream(a, a, 16, 16, 4)
    with pytest.raises(ValueError):
        lbm.lbm_probe_stream(a[:10], b, 16, 16, 4)

"""GPU check of rr_stencil2d (Sec. III.D) against the fp64 oracle within the
fp32 rounding bound (n + 2) * 2^-24 * sum |w x| per point; edge points exact."""
import numpy as np
import pytest

import rr_synth
from tests.test_emulated_kernels import STENCIL_GRIDS_SMALL, check_stencil

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    import torch
    import paper_1011_3583_amd as rr
    assert torch.cuda.is_available()
    rr.lib()
    return rr


def gpu_stencil(rr, x, radius, weights, shape=0):
    import torch
    print(f"stencil {x.shape} r={radius} shape={shape}", flush=True)
    src = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    dst = torch.empty_like(src)
    st = rr.stencil2d_raw(dst.data_ptr(), src.data_ptr(), x.shape[0], x.shape[1], radius, weights, shape,
                          torch.cuda.current_stream().cuda_stream)
    assert st == 0, rr.last_error()
    torch.cuda.synchronize()
    return dst.cpu().numpy()


def test_stencil_fd_orders_small_grids(rr):
    g = rr_synth.rng(17)
    for t, (rows, cols) in enumerate(STENCIL_GRIDS_SMALL):
        x = rr_synth.random_grid(300 + t, rows, cols)
        for r, c in rr_synth.FD_LAPLACIAN.items():
            check_stencil(gpu_stencil(rr, x, r, c), x, r, c, 0)
        r = int(g.integers(1, 5))
        w = g.uniform(-1, 1, (2 * r + 1) ** 2).astype(np.float32)
        check_stencil(gpu_stencil(rr, x, r, w, 1), x, r, w, 1)


def test_stencil_paper_grid_4096(rr):
    """Table 4's data set: 4096 x 4096 floats, FD orders I-IV and a 5x5 box."""
    x = rr_synth.random_grid(4096, 4096, 4096)
    for r, c in rr_synth.FD_LAPLACIAN.items():
        check_stencil(gpu_stencil(rr, x, r, c), x, r, c, 0)
    w = rr_synth.rng(5).uniform(-1, 1, 25).astype(np.float32)
    check_stencil(gpu_stencil(rr, x, 2, w, 1), x, 2, w, 1)


def test_stencil_grid_above_2_24_points(rr):
    """A grid just above 2^24 points takes the 16-row tiles (smaller grids take
    32-row tiles): FD orders I and IV and a 3x3 box against the oracle."""
    x = rr_synth.random_grid(4100, 4100, 4100)
    for r in (1, 4):
        c = rr_synth.FD_LAPLACIAN[r]
        check_stencil(gpu_stencil(rr, x, r, c), x, r, c, 0)
    w = rr_synth.rng(6).uniform(-1, 1, 9).astype(np.float32)
    check_stencil(gpu_stencil(rr, x, 1, w, 1), x, 1, w, 1)


def test_stencil_polynomial_field(rr):
    """The order-I Laplacian of i^2 + j^2 is exactly 4 in fp32 (exact weights, exact
    sums of integers below 2^24)."""
    rows, cols = 1000, 1500
    i = np.arange(rows, dtype=np.float64)[:, None]
    j = np.arange(cols, dtype=np.float64)[None, :]
    x = (i ** 2 + j ** 2).astype(np.float32)
    out = gpu_stencil(rr, x, 1, rr_synth.FD_LAPLACIAN[1])
    assert np.array_equal(out[1:-1, 1:-1], np.full((rows - 2, cols - 2), 4.0, dtype=np.float32))

"""The pull-only copy (fslbm_pull_copy_time, the memory bound of the
stream-collide): through the C ABI on a ragged periodic lattice, every
plane must hold dst_q(x) = src_q(x - c_q) bit for bit, for each element
size, and the gap between planes must stay untouched."""
import numpy as np
import pytest

from paper_1509_07691_amd import fslbm as F

pytestmark = pytest.mark.gpu

# the library's direction order (q-major planes): rest, the six faces, then
# the twelve edges in opposite pairs
C = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
     (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


@pytest.mark.parametrize("precision,elem", [(F.FSLBM_F64, 8), (F.FSLBM_F32, 4), (F.FSLBM_F16_STORE, 2),
                                            (F.FSLBM_BF16_STORE, 2)])
def test_pull_copy_moves_every_value_from_upstream(precision, elem):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    nx, ny, nz = 13, 17, 19
    n = nx * ny * nz
    nbytes = F.fslbm_pull_copy_bytes(nx, ny, nz, precision)
    ns = nbytes // (19 * elem)
    dt = {8: torch.int64, 4: torch.int32, 2: torch.int16}[elem]
    g = torch.Generator().manual_seed(3)
    src = torch.randint(-2 ** 15, 2 ** 15, (19 * ns,), generator=g, dtype=torch.int64).to(dt).cuda()
    sentinel = 0x5A5A
    dst = torch.full((19 * ns,), sentinel, dtype=dt, device="cuda")
    torch.cuda.synchronize()
    us = F.fslbm_pull_copy_time(nx, ny, nz, precision, src.data_ptr(), dst.data_ptr(), nbytes,
                                torch.cuda.current_stream().cuda_stream, 3)
    torch.cuda.synchronize()
    print(f"precision {precision}: {us:.2f} us per launch on {nx}x{ny}x{nz}")
    assert us > 0.0
    s = src.cpu().numpy().reshape(19, ns)
    d = dst.cpu().numpy().reshape(19, ns)
    for q, (cx, cy, cz) in enumerate(C):
        expect = np.roll(s[q, :n].reshape(nz, ny, nx), shift=(cz, cy, cx), axis=(0, 1, 2))
        assert np.array_equal(d[q, :n].reshape(nz, ny, nx), expect), q
        assert (d[q, n:] == sentinel).all(), q

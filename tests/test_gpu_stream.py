"""The two streaming references the step's bandwidth is measured against:
lbfz_stream_copy moves every byte unchanged, and lbfz_stream_planes moves
plane k of every node to the row k mod 3 selects (one row down, in place,
one row up; y periodic) -- checked element by element on distinct values,
with a ragged grid and a plane stride larger than a plane."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_stream_copy_moves_every_byte():
    import torch
    from paper_2511_09422_amd.lbfz import lbfz_stream_copy
    n = 4 * 1000003
    a = torch.arange(n, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    lbfz_stream_copy(b.data_ptr(), a.data_ptr(), 4 * n, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("nx,ny", [(64, 48), (77, 5), (1, 3)])
def test_stream_planes_pattern(nx, ny):
    import torch
    from paper_2511_09422_amd.lbfz import lbfz_stream_planes
    N = nx * ny
    ps = N + 37
    src = np.random.default_rng(nx * ny).standard_normal(30 * ps).astype(np.float32)
    a = torch.tensor(src, device="cuda")
    b = torch.full_like(a, np.nan)
    lbfz_stream_planes(b.data_ptr(), a.data_ptr(), nx, ny, ps,
                       torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = b.cpu().numpy()
    for k in range(30):
        plane = src[k * ps:k * ps + N].reshape(ny, nx)
        want = np.roll(plane, (k % 3) - 1, axis=0)   # row y lands on y - 1, y, y + 1
        assert np.array_equal(got[k * ps:k * ps + N].reshape(ny, nx), want), k
        assert np.isnan(got[k * ps + N:(k + 1) * ps]).all()   # padding untouched

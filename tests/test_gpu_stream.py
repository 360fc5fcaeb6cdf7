"""The streaming references the steps' bandwidth is measured against:
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


CX19 = [0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0]
CY19 = [0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1]
CZ19 = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1]


@pytest.mark.parametrize("nx,ny,nz,nread,nwrite", [(5, 4, 3, 22, 5), (7, 3, 4, 50, 42),
                                                   (1, 2, 3, 50, 42)])
def test_stream_planes3d_pattern(nx, ny, nz, nread, nwrite):
    """lbfz_stream_planes3d moves plane k < 38 of every node to the node one
    D3Q19 direction (k mod 19) away (periodic in x, y, z) and the planes from
    38 on in place -- element by element on distinct values, ragged grids, a
    plane stride larger than a plane; the padding is untouched."""
    import torch
    from paper_2511_09422_amd.lbfz import lbfz_stream_planes3d
    N = nx * ny * nz
    ps = N + 29
    src = np.random.default_rng(N + nread).standard_normal(nread * ps).astype(np.float32)
    a = torch.tensor(src, device="cuda")
    b = torch.full((nwrite * ps,), float("nan"), dtype=torch.float32, device="cuda")
    lbfz_stream_planes3d(b.data_ptr(), a.data_ptr(), nx, ny, nz, ps, nread, nwrite,
                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = b.cpu().numpy()
    for k in range(nwrite):
        plane = src[k * ps:k * ps + N].reshape(nz, ny, nx)
        d = k % 19
        want = np.roll(plane, (CZ19[d], CY19[d], CX19[d]), axis=(0, 1, 2)) if k < 38 else plane
        assert np.array_equal(got[k * ps:k * ps + N].reshape(nz, ny, nx), want), k
        assert np.isnan(got[k * ps + N:(k + 1) * ps]).all()


def test_stream_planes3d_rejects_bad_counts():
    import torch
    from paper_2511_09422_amd import lbfz
    a = torch.zeros(64, device="cuda")
    for nr, nw in ((0, 1), (51, 5), (22, 6), (50, 41), (5, 5)):
        with pytest.raises(lbfz.LbfzError):
            lbfz.lbfz_stream_planes3d(a.data_ptr(), a.data_ptr(), 2, 2, 2, 8, nr, nw, 0)

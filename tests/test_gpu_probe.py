"""GPU checks of the measurement references.  The reference read
(pamx_read_probe), the plain read of a matrix in the SWAP pass's launch shape
that the benchmark times beside the pass: every work-group's sum equals the
sum of the block it was given
(1024-column tiles, row chunks, ragged last tile and chunk, columns read up
to the next multiple of 4; chunks of 4096 rows and more take the pass's
prefetching loop).  The reference store (pamx_write_probe), the distance
kernel's stores alone: every entry written, the padding untouched."""
import pytest

from paper_2008_05171_amd import pamx as abi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("n,chunk", [(1, 1), (2101, 300), (3000, 1000), (1500, 7), (5000, 4096),
                                     (4100, 4100)])
def test_read_probe_block_sums(n, chunk):
    print("[case] read_probe", n, chunk, flush=True)
    ld = (n + 3) // 4 * 4 + 4                      # padded row stride
    g = torch.Generator().manual_seed(n)
    base = torch.rand(n, ld, generator=g, dtype=torch.float32)
    D = base.to(DEV)[:, :n]
    tiles, q = (n + 1023) // 1024, (n + chunk - 1) // chunk
    sums = torch.full((tiles * q,), -1.0, dtype=torch.float32, device=DEV)
    abi.pamx_read_probe(D, chunk, sums)
    torch.cuda.synchronize()
    got = sums.cpu().double().view(q, tiles)
    cols = (n + 3) // 4 * 4
    b64 = base.double()
    for y in range(q):
        for x in range(tiles):
            blk = b64[y * chunk:min((y + 1) * chunk, n), x * 1024:min((x + 1) * 1024, cols)]
            want = blk.sum().item()
            # FP32 sums: each lane adds 4 values per row of the chunk
            tol = max(1e-4, 4.0 * blk.shape[0] * 2.0 ** -24) * max(1.0, want)
            assert abs(got[y, x].item() - want) <= tol, (y, x, got[y, x], want)


@pytest.mark.parametrize("n,ld", [(1, 4), (63, 64), (1000, 1003), (1537, 1600)])
def test_write_probe_covers_the_matrix(n, ld):
    """pamx_write_probe writes its value to every entry (r, c < n) and leaves
    the padding columns alone (ragged tiles, padded and odd strides)."""
    print("[case] write_probe", n, ld, flush=True)
    buf = torch.full((n, ld), -3.0, dtype=torch.float32, device=DEV)
    abi.pamx_write_probe(buf[:, :n], 2.5, ld=ld)
    torch.cuda.synchronize()
    got = buf.cpu()
    assert bool((got[:, :n] == 2.5).all())
    assert bool((got[:, n:] == -3.0).all())

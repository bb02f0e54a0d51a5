"""The ceiling probes the benchmark uses: the FP32 atomic-add probe adds
exactly once per valid address and launch (counts are exact in FP32 at these
sizes) and skips addresses outside the grid; the copy probe copies."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_atomic_probe_counts_every_add(eng, N):
    import torch
    cells, n, reps = 4096, 1 << 16, 3
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    addr = torch.randint(-16, cells + 16, (n,), generator=g, device="cuda", dtype=torch.int32)
    grid = torch.zeros(cells, dtype=torch.float32, device="cuda")
    ms = N.psl_probe_atomics(grid.data_ptr(), cells, addr.data_ptr(), n, reps)
    torch.cuda.synchronize()
    assert ms > 0
    a = addr.cpu().numpy()
    valid = a[(a >= 0) & (a < cells)]
    expect = np.bincount(valid, minlength=cells).astype(np.float64) * (reps + 1)  # + warm-up
    assert np.array_equal(grid.cpu().numpy().astype(np.float64), expect)


def test_copy_probe_copies(eng, N):
    import torch
    nbytes = 1 << 20
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    ms = N.psl_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, 2)
    torch.cuda.synchronize()
    assert ms > 0
    assert torch.equal(dst, src)


def test_probes_reject_bad_sizes(eng, N):
    import torch
    grid = torch.zeros(16, dtype=torch.float32, device="cuda")
    addr = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(N.PslError):
        N.psl_probe_atomics(grid.data_ptr(), 0, addr.data_ptr(), 16, 1)
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.PslError):
        N.psl_probe_copy(a.data_ptr(), a.data_ptr(), 15, 1)

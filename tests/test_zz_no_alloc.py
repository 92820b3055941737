"""The allocation-free device aggregation (sa_aggregate_device_noalloc) against the
allocating entry point sa_aggregate_device, through the C ABI: two calls in a row, the
second on a smaller graph, results bit for bit equal.  A caller allocator that refuses
every request is installed during the allocation-free calls, so any device allocation
by the library would fail them."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2606_24748_amd import blkamg as B  # noqa: E402
from tests.gpu_util import q1_problem, to_device_bsr  # noqa: E402


def _refusing_allocator(log):
    def alloc(nbytes, _ctx):
        log.append(int(nbytes))
        return None  # the library turns this into ENOMEM

    def free(_ptr, _nbytes, _ctx):
        log.append(-1)

    return alloc, free


@pytest.mark.parametrize("seed", [3, 0x1234])
def test_noalloc_aggregation_matches_allocating_entry_point(seed):
    for n in (12, 7):  # the second graph is smaller than the first
        print(f"no-alloc aggregation n={n} seed={seed:#x}", flush=True)
        m, i, j, v, A = q1_problem(n, mat_seed=5)
        H, keep = to_device_bsr(A)
        want, na_w, nr_w = B.sa_aggregate_device(H, m.dirichlet, seed=seed)
        d_dir = torch.as_tensor(m.dirichlet.astype(np.uint8)).cuda()
        got = torch.full((m.n_nodes,), -7, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        log = []
        B.blkamg_set_allocator(*_refusing_allocator(log))
        try:
            na, nr = B.sa_aggregate_device_noalloc(H, d_dir, got, seed=seed)
        finally:
            B.blkamg_set_allocator()
        assert log == [], f"the allocation-free call asked the allocator for {log}"
        assert (na, nr) == (na_w, nr_w)
        assert torch.equal(got, want)
        # every non-Dirichlet vertex aggregated, ids 0..n_agg-1 all used
        g = got.cpu().numpy()
        assert np.all((g >= 0) == ~m.dirichlet.astype(bool))
        assert np.array_equal(np.unique(g[g >= 0]), np.arange(na))


def test_noalloc_aggregation_refuses_graphs_beyond_the_scratch():
    """A graph whose scratch would exceed the static array is refused before any launch."""
    n = 2_400_000
    rp = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.arange(n, dtype=torch.int32, device="cuda")
    val = torch.ones(n, 1, 1, dtype=torch.float64, device="cuda")
    H = B.bsr_create(n, n, 1, 1, rp, ci, val)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BlkAmgError) as e:
        B.sa_aggregate_device_noalloc(H, None, out)
    assert e.value.code == B.EINVAL and "static scratch" in str(e.value)
    # just below the limit the call runs (isolated vertices: one aggregate each)
    small = 2_000_000
    H2 = B.bsr_create(small, small, 1, 1, rp[:small + 1].contiguous(), ci[:small].contiguous(), val[:small].contiguous())
    na, nr = B.sa_aggregate_device_noalloc(H2, None, out[:small])
    assert na == small and nr == 1
    assert torch.equal(out[:small], torch.arange(small, dtype=torch.int32, device="cuda"))

"""kc_scratch_bytes against what kc_reserve really allocates on the device
(free device memory before and after, within the allocator's rounding)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2305_07545_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load_library()


@pytest.mark.parametrize("X,Y,n,alpha,k_h", [(2621, 2657, 150_000_000, 8, 1),
                                             (2621, 2657, 20_000_000, 5, 3),
                                             (31627, 31657, 60_000_000, 8, 1)])
def test_scratch_bytes_is_what_reserve_allocates(X, Y, n, alpha, k_h):
    print(f"case sizing X={X} Y={Y} n={n} alpha={alpha} k_h={k_h}", flush=True)
    words = torch.empty(X * Y, dtype=torch.int64, device="cuda")
    bf = P.CountBF(X, Y, alpha, k_h, words=words)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    bf.reserve(n)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    used = free0 - free1
    want = P.scratch_bytes(X, Y, n, alpha, k_h) - 256  # the status word came with the handle
    bf.close()
    assert abs(used - want) <= 64 * 2**20 + 0.02 * want, (used, want)

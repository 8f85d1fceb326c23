"""The allocation-free forward entry point of the learned-screen model against
the allocating one, through the C ABI: bit-identical outputs on two calls in a
row (the second with fewer rows, so stale scratch rows of the first call must
not leak into it), the row limit rejected, and no device allocation by the
calls after the first on the device (the caching allocator's counters and the
device's free memory stay put)."""
import numpy as np
import pytest

from paper_2604_10743_amd import synth

pytestmark = pytest.mark.gpu


def test_mlp_forward_noalloc_matches_forward():
    import torch
    import paper_2604_10743_amd as P
    assert torch.cuda.is_available()
    m = P.MLP(synth.init_mlp_params(21, out_bias=0.2))
    rng = np.random.default_rng(3)
    nmax = P.MLP.noalloc_max_rows()
    assert nmax == 4096
    # the first call on a device looks the array up (the runtime materialises
    # the module's device globals then); the calls after it allocate nothing
    X1 = torch.zeros((1, 16), device="cuda")
    y1 = torch.zeros(1, device="cuda")
    m.forward_noalloc(X1, y1)
    torch.cuda.synchronize()
    for n in (3000, 257):                      # second call smaller than the first
        X = torch.as_tensor(rng.standard_normal((n, 16)).astype(np.float32), device="cuda")
        y = torch.full((n,), float("nan"), device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        alloc0 = torch.cuda.memory_stats().get("num_alloc_retries", 0), torch.cuda.memory_allocated()
        m.forward_noalloc(X, y)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert (torch.cuda.memory_stats().get("num_alloc_retries", 0), torch.cuda.memory_allocated()) == alloc0
        ref = m.forward(X)
        a, b = y.cpu().numpy(), ref.cpu().numpy()
        print(f"noalloc n={n}: max |dy| = {np.max(np.abs(a - b)):.3e}", flush=True)
        assert np.all(np.isfinite(a)) and np.array_equal(a, b)
    # the limit: one row too many is an error, the maximum works
    Xb = torch.zeros((nmax + 1, 16), device="cuda")
    yb = torch.zeros(nmax + 1, device="cuda")
    with pytest.raises(P.EmError):
        m.forward_noalloc(Xb, yb)
    m.forward_noalloc(Xb[:nmax], yb[:nmax])
    torch.cuda.synchronize()
    assert np.array_equal(yb[:nmax].cpu().numpy(), m.forward(Xb[:nmax]).cpu().numpy())
    m.close()

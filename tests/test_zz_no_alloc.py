"""The allocation-free variant of the cost-model forward/backward (for callers that
cannot allocate: graph capture, tight training loops) against the allocating entry
point, on two calls in a row, the second with a smaller batch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _noalloc(F, B, p, X, t, y, g, loss):
    """Through the C ABI, on the current stream; returns the status."""
    from paper_2108_03991_amd import slim
    try:
        slim.mlp_forward_backward_noalloc(F, B, p, X, t, y, g, loss)
        return 0
    except slim.SlimError as e:
        return e.code


def test_noalloc_matches_allocating_entry_point():
    import torch
    from paper_2108_03991_amd import slim
    F = 5
    npar = 64 * F + 64 + 64 * 64 + 64 + 64 + 1
    rng = np.random.default_rng(7)
    p = torch.tensor(rng.standard_normal(npar).astype(np.float32) * 0.3, device='cuda')
    for B in (5000, 700):                       # the second call is smaller: stale workspace must not leak in
        X = torch.tensor(rng.standard_normal((B, F)).astype(np.float32), device='cuda')
        t = torch.tensor(rng.standard_normal(B).astype(np.float32), device='cuda')
        ref = [torch.zeros(B, device='cuda'), torch.zeros(npar, device='cuda'), torch.zeros(1, device='cuda')]
        got = [torch.full((B,), 7.0, device='cuda'), torch.full((npar,), 7.0, device='cuda'),
               torch.full((1,), 7.0, device='cuda')]
        slim.mlp_forward_backward(F, B, p, X, t, *ref)
        assert _noalloc(F, B, p, X, t, *got) == 0
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        assert float(ref[2]) > 0 and torch.isfinite(ref[1]).all()
    # beyond the workspace: a clear argument error, nothing launched
    big = 32768 + 1
    dummy = torch.zeros(1, device='cuda')
    assert _noalloc(F, big, p, dummy, dummy, dummy, dummy, dummy) == 1

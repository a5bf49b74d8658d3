"""GPU forward/backward of the cost-model network vs the FP64 oracle backprop."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _pack(p):
    return np.concatenate([p['W1'].ravel(), p['b1'], p['W2'].ravel(), p['b2'], p['w3'], p['b3']]).astype(np.float32)


@pytest.mark.parametrize("B", [1, 63, 200])
def test_gradients_match_oracle(B):
    import torch
    from paper_2108_03991_amd import slim
    F = 5
    rng = np.random.default_rng(B)
    p = mlp.init_params(F, seed=3)
    p['b1'] = rng.standard_normal(64) * 0.1
    p['b2'] = rng.standard_normal(64) * 0.1
    X = rng.standard_normal((B, F))
    t = rng.standard_normal(B)
    # evaluate the oracle at the FP32-rounded parameters and inputs
    p32 = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    X32 = X.astype(np.float32).astype(np.float64)
    t32 = t.astype(np.float32).astype(np.float64)
    loss_ref, g_ref = mlp.loss_and_grad(p32, X32, t32)
    y_ref, _ = mlp.forward(p32, X32)
    dev = 'cuda'
    P = torch.tensor(_pack(p32), device=dev)
    Xt = torch.tensor(X32.astype(np.float32), device=dev)
    Tt = torch.tensor(t32.astype(np.float32), device=dev)
    y = torch.zeros(B, dtype=torch.float32, device=dev)
    grad = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    slim.mlp_forward_backward(F, B, P, Xt, Tt, y, grad, loss)
    torch.cuda.synchronize()
    gr = _pack(g_ref).astype(np.float64)
    gg = grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gg - gr) <= 1e-4 * np.linalg.norm(gr)
    assert np.abs(y.cpu().numpy() - y_ref).max() <= 1e-4 * max(1.0, np.abs(y_ref).max())
    assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref

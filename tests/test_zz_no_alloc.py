"""dvm_mlp_gradient_noalloc (static device scratch, no allocation, no
workspace) against dvm_mlp_gradient (bound workspace) through the C
interface: two calls in a row, the second with a smaller batch, give the
same loss and gradients bitwise; batches beyond the static limit are refused."""
import numpy as np
import pytest

from paper_1503_00707_amd import dvm as D
from paper_1503_00707_amd import inputs as I

pytestmark = pytest.mark.gpu


def _data(seed, n):
    rng = np.random.default_rng(seed)
    p = I.mlp_init(seed).astype(np.float32)
    p[:I.MLP_WEIGHTS] += rng.normal(0, 0.05, I.MLP_WEIGHTS).astype(np.float32)
    p[I.MLP_WEIGHTS:I.MLP_WEIGHTS + 10] = rng.normal(0, 0.3, 10)
    p[I.MLP_WEIGHTS + 10:] = rng.uniform(0.5, 2.0, 10)
    x = rng.normal(0, 1.0, (n, 10)).astype(np.float32)
    y = (rng.random(n) < 0.3).astype(np.float32)
    return p, x, y


def test_noalloc_gradient_equals_workspace_gradient_twice():
    import torch
    print("no-alloc gradient: batches 8192 then 701", flush=True)
    grad = torch.empty(I.MLP_WEIGHTS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    for seed, n in ((1, 8192), (2, 701)):
        p, x, y = _data(seed, n)
        xt, yt = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
        net = D.MLP(p, max_batch=8192)
        net.gradient(xt, yt, pos_weight=2.5)
        g_ref, l_ref = net.grads_and_loss()
        D.mlp_gradient_noalloc(net.params, xt, yt, pos_weight=2.5, grad=grad, loss=loss)
        torch.cuda.synchronize()
        assert np.array_equal(grad.cpu().numpy(), g_ref.cpu().numpy()), n
        assert float(loss.item()) == l_ref, n
        assert np.abs(g_ref.cpu().numpy()).max() > 0


def test_noalloc_gradient_refuses_batches_beyond_its_scratch():
    import torch
    p, x, y = _data(3, 16)
    pt = torch.as_tensor(p).cuda()
    big = torch.zeros((8193, 10), dtype=torch.float32, device="cuda")
    yb = torch.zeros(8193, dtype=torch.float32, device="cuda")
    with pytest.raises(D.DvmError) as e:
        D.mlp_gradient_noalloc(pt, big, yb)
    assert e.value.code == D.ERR_WORKSPACE
    with pytest.raises(D.DvmError):
        D.mlp_gradient_noalloc(pt, big[:0], yb[:0])
    torch.cuda.synchronize()

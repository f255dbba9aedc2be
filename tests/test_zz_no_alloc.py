"""The entry point that allocates nothing (mlp_grad_noalloc, snake_mlp.h):
called through the C ABI twice in a row, the second call with a smaller
batch, its gradient and loss equal mlp_grad's (the same kernels on the same
inputs give the same bits); batches beyond its fixed scratch are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
snk = pytest.importorskip("paper_1904_02833_amd")


def net_and_data(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=0.1, size=6467).astype(np.float32)
    ms = np.concatenate([rng.normal(size=32), rng.uniform(0.5, 2.0, size=32)]).astype(np.float32)
    net = snk.Net(p, ms)
    x = torch.as_tensor(rng.normal(size=(n, 32)).astype(np.float32), device="cuda")
    t = torch.as_tensor(rng.normal(size=(n, 3)).astype(np.float32), device="cuda")
    return net, x, t


def test_noalloc_grad_equals_grad_on_two_calls():
    for n, seed in ((4096, 1), (1000, 2)):
        net, x, t = net_and_data(n, seed)
        g_ref, l_ref = net.grad(x, t)
        g, l = net.grad_noalloc(x, t)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), n
        assert torch.equal(l, l_ref), n
        print(f"\n[noalloc] n={n} loss {float(l):.6g} max|g| {float(g.abs().max()):.3g}")


def test_noalloc_refuses_batches_beyond_its_scratch():
    net, x, t = net_and_data(4097, 3)
    with pytest.raises(snk.SimError) as e:
        net.grad_noalloc(x, t)
    assert "4096" in str(e.value)

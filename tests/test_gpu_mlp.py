"""Warm-start network kernels (BF16 MFMA, FP32 accumulation) against the FP64
oracle.

The oracle receives the parameters already rounded to BF16 (the operands the
GPU multiplies) and evaluates everything else in FP64.  The GPU additionally
rounds each activation to BF16 before it enters a product (relative half-ulp
u = 2^-9); through three layers this bounds the output error by a few u of
the output scale, and the gradients by about ten u of their norm.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
snk = pytest.importorskip("paper_1904_02833_amd")

U = 2.0 ** -9


def bf16_round(a):
    t = torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32)
    return t.numpy().astype(np.float64)


def bf16_weights(p):
    """Round the weight matrices (not the biases) as the GPU does."""
    q = np.array(p, np.float64)
    for a, b in ((0, 2048), (2112, 6208), (6272, 6464)):
        q[a:b] = bf16_round(q[a:b])
    return q


def setup(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=0.25, size=6467).astype(np.float32)
    x = (rng.normal(size=(n, 32)) * rng.uniform(0.5, 3, 32) + rng.normal(size=32)).astype(np.float32)
    t = rng.normal(size=(n, 3)).astype(np.float32)
    return p, x, t


@pytest.mark.parametrize("n", [1, 64, 1000, 4096 + 13])
def test_forward_matches_oracle(n):
    p, x, t = setup(n, 10 + n)
    xd = torch.as_tensor(x, device="cuda")
    ms = snk.Net.norm_stats(xd)
    mean, std = oracle.mlp_norm_stats(x.astype(np.float64))
    msh = ms.cpu().numpy()
    assert np.allclose(msh[:32], mean, rtol=1e-6, atol=1e-6)
    assert np.allclose(msh[32:], std, rtol=1e-5)
    net = snk.Net(p, ms)
    y = net.forward(xd).cpu().numpy().astype(np.float64)
    yo = oracle.mlp_forward(bf16_weights(p), msh[:32], msh[32:], x)
    scale = np.abs(yo).max()
    err = np.abs(y - yo).max()
    print(f"\n[mlp fwd n={n}] max err {err:.3g} scale {scale:.3g} ({err / scale / U:.2f} u)")
    assert err <= 8 * U * scale


GRAD_K = 12


def test_gradient_matches_oracle():
    """Every gradient entry against the FP64 oracle (BF16-rounded weights),
    within GRAD_K unit roundoffs of its own error scale A (the oracle's sum
    over samples of |delta| |activation| for that entry, deltas carried back
    through absolute values): the kernel rounds each activation and each
    delta to BF16 before it enters a product (u each) and the forward and
    backward errors of those operands are a few u of the same scale.  A
    sign error in the largest entry of any parameter group would exceed the
    bound (checked), so the gate is element-wise, not a norm."""
    n = 2000
    p, x, t = setup(n, 3)
    xd, td = torch.as_tensor(x, device="cuda"), torch.as_tensor(t, device="cuda")
    ms = snk.Net.norm_stats(xd)
    msh = ms.cpu().numpy().astype(np.float64)
    net = snk.Net(p, ms)
    g, loss = net.grad(xd, td)
    g = g.cpu().numpy().astype(np.float64)
    pb = bf16_weights(p)
    lo, go = oracle.mlp_loss_grad(pb, msh[:32], msh[32:], x, t)
    A = oracle.mlp_grad_abs(pb, msh[:32], msh[32:], x, t)
    assert abs(float(loss.cpu()) - lo) <= 1e-2 * lo
    floor = 1e-12 * A.max()
    for name, a, b in (("W1", 0, 2048), ("b1", 2048, 2112), ("W2", 2112, 6208), ("b2", 6208, 6272),
                       ("W3", 6272, 6464), ("b3", 6464, 6467)):
        err = np.abs(g[a:b] - go[a:b])
        ratio = err / (U * A[a:b] + floor)
        rel = np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
        k = int(np.argmax(np.abs(go[a:b])))
        print(f"[mlp grad] {name}: worst entry {ratio.max():.3g} u of its scale "
              f"(entry {int(np.argmax(ratio))}), norm-relative {rel:.3g}", flush=True)
        assert ratio.max() <= GRAD_K, name
        assert 2 * abs(go[a + k]) > GRAD_K * U * A[a + k], name
    # deterministic: the same call twice gives the same bits
    g2, _ = net.grad(xd, td)
    assert np.array_equal(g2.cpu().numpy().astype(np.float64), g)


def test_adam_matches_oracle():
    rng = np.random.default_rng(5)
    p = rng.normal(size=6467).astype(np.float32)
    ms = torch.cat([torch.zeros(32), torch.ones(32)]).cuda()
    net = snk.Net(p, ms)
    po = p.astype(np.float64)
    m, v = np.zeros(6467), np.zeros(6467)
    for step in range(1, 6):
        g = rng.normal(size=6467).astype(np.float32)
        net.adam(torch.as_tensor(g, device="cuda"), lr=1e-2)
        oracle.mlp_adam(po, m, v, g.astype(np.float64), step, lr=1e-2)
    got = net.params.cpu().numpy().astype(np.float64)
    assert np.abs(got - po).max() <= 1e-5


def test_training_reduces_loss():
    """Fit a smooth map of the inputs with the GPU kernels only."""
    rng = np.random.default_rng(7)
    n = 8192
    x = rng.normal(size=(n, 32)).astype(np.float32)
    t = np.stack([np.tanh(x[:, 0] + 0.5 * x[:, 1]), x[:, 2] * x[:, 3] * 0.3,
                  np.sin(x[:, 4])], 1).astype(np.float32)
    xd, td = torch.as_tensor(x, device="cuda"), torch.as_tensor(t, device="cuda")
    ms = snk.Net.norm_stats(xd)
    net = snk.Net((rng.normal(size=6467) * 0.1).astype(np.float32), ms)
    _, l0 = net.grad(xd, td)
    for it in range(300):
        idx = torch.as_tensor(rng.integers(0, n, 1024), device="cuda")
        g, _ = net.grad(xd[idx].contiguous(), td[idx].contiguous())
        net.adam(g, lr=3e-3)
    _, l1 = net.grad(xd, td)
    print(f"\n[mlp train] loss {float(l0.cpu()):.4f} -> {float(l1.cpu()):.4f}")
    assert float(l1.cpu()) < 0.2 * float(l0.cpu())

"""GPU parity of the surrogate-network kernels (BF16 matrix-core products, FP32 accumulation)
against the FP64 CPU network in oracle/mlp_oracle.py, through the C ABI.

Tolerances follow from the arithmetic: operands are rounded to BF16 (unit roundoff 2^-9 = 2e-3)
before every product, accumulation is FP32.  A single affine layer with operands that are exact in
BF16 and sums exact in FP32 must match bit for bit (this pins the matrix-core lane layout and the
tile edges); deeper networks carry one BF16 rounding per layer, so the output is compared at
rel-L2 <= 2e-2 and the gradients at rel-L2 <= 3e-2 per parameter block.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
M = O.mlp_oracle


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def fpn():
    import paper_2106_08040_amd as fpn
    return fpn


@pytest.fixture(scope="module")
def ctx(fpn):
    import torch
    assert torch.cuda.is_available()
    c = fpn.Context(0)
    yield c
    c.close()


def _exact_layer(fpn, ctx, n, k, out, seed):
    """One affine layer whose operands are small multiples of 1/8: exact in BF16, sums exact in FP32."""
    import torch
    r = np.random.default_rng(seed)
    net = fpn.MLP(ctx, [k, out], seed=seed)
    W = r.integers(-8, 9, size=(out, k)) / 8.0
    b = r.integers(-8, 9, size=out) / 8.0
    net.set_params(np.concatenate([W.ravel(), b]))
    x = r.integers(-4, 5, size=(n, k)).astype(np.float64)
    return net, W, b, x


@pytest.mark.parametrize("n,k,out", [(64, 32, 32), (200, 256, 96), (1000, 512, 256)])
def test_single_layer_is_exact(fpn, ctx, n, k, out):
    import torch
    net, W, b, x = _exact_layer(fpn, ctx, n, k, out, seed=n + k)
    y = net.forward(x).cpu().numpy()
    ref, _ = M.forward([W], [b], x)
    assert np.array_equal(y.astype(np.float64), ref), np.abs(y - ref).max()
    net.close()


def test_single_layer_weight_gradient_is_exact(fpn, ctx):
    """dW = dz^T x with dz = 2 (y - t) / (n out): targets t = y - delta (delta a small integer, y from the
    reference) and n out = 2048 keep every dz and every sum exact in BF16 / FP32."""
    n, k, out = 64, 64, 32
    net, W, b, x = _exact_layer(fpn, ctx, n, k, out, seed=5)
    r = np.random.default_rng(6)
    y, cache = M.forward([W], [b], x)
    t = y - r.integers(-2, 3, size=(n, out))
    g, loss = net.gradient(x, t)
    g = g.cpu().numpy().astype(np.float64)
    gW, gb = M.backward([W], cache, y, t)
    assert np.array_equal(g[:out * k].reshape(out, k), gW[0])
    assert np.array_equal(g[out * k:], gb[0])
    assert abs(float(loss.item()) - M.loss(y, t)) <= 1e-12 * M.loss(y, t)
    net.close()


PROD = [8, 512, 512, 512, 512, 256]


@pytest.mark.parametrize("n", [1, 300, 4096])
def test_production_network_forward(fpn, ctx, n):
    net = fpn.MLP(ctx, PROD, seed=11)
    assert net.n_params == 923904
    r = np.random.default_rng(n)
    x = r.normal(size=(n, 8))
    mean, std = r.normal(size=8) * 0.1, r.uniform(0.5, 2.0, 8)
    net.set_input_norm(mean, std)
    y = net.forward(x).cpu().numpy()
    Ws, bs = net.unflatten(net.get_params().cpu().numpy().astype(np.float64))
    ref, _ = M.forward(Ws, bs, (x - mean.astype(np.float32)) / std.astype(np.float32))
    e = rel(y, ref)
    print(f"forward n={n}: rel-L2 {e:.2e}", flush=True)
    assert e < 2e-2
    net.close()


def test_production_network_gradient(fpn, ctx):
    net = fpn.MLP(ctx, PROD, seed=12)
    r = np.random.default_rng(3)
    n = 777
    x = r.normal(size=(n, 8))
    t = r.normal(size=(n, 256)) * 0.3
    g, loss = net.gradient(x, t)
    g = g.cpu().numpy().astype(np.float64)
    Ws, bs = net.unflatten(net.get_params().cpu().numpy().astype(np.float64))
    y, cache = M.forward(Ws, bs, x)
    gW, gb = M.backward(Ws, cache, y, t)
    assert abs(float(loss.item()) - M.loss(y, t)) < 2e-2 * M.loss(y, t)
    gWg, gbg = net.unflatten(g)
    for l in range(len(Ws)):
        ew, eb = rel(gWg[l], gW[l]), rel(gbg[l], gb[l])
        print(f"layer {l}: dW {ew:.2e} db {eb:.2e}", flush=True)
        assert ew < 3e-2 and eb < 3e-2
    net.close()


def test_adam_step_matches_oracle_update(fpn, ctx):
    """One Adam step on the device equals the reference update applied to the device's own gradient."""
    net = fpn.MLP(ctx, [8, 64, 32], seed=13)
    r = np.random.default_rng(4)
    import torch
    x = torch.as_tensor(r.normal(size=(100, 8)), dtype=torch.float32, device="cuda:0")
    t = torch.as_tensor(r.normal(size=(100, 32)), dtype=torch.float32, device="cuda:0")
    p0 = net.get_params().cpu().numpy().astype(np.float64)
    g, _ = net.gradient(x, t)
    g = g.cpu().numpy().astype(np.float64)
    net.train_step(x, t, 1e-3)
    p1 = net.get_params().cpu().numpy().astype(np.float64)
    ref = p0.copy()
    M.adam_step([ref], [g], [np.zeros_like(ref)], [np.zeros_like(ref)], 1, lr=1e-3)
    assert np.abs(p1 - ref).max() < 1e-6
    net.close()


def test_training_reduces_loss(fpn, ctx):
    """A smooth synthetic map is learned: the loss falls by more than 10x in 300 Adam steps."""
    import torch
    net = fpn.MLP(ctx, [8, 128, 128, 64], seed=14)
    r = np.random.default_rng(8)
    X = r.uniform(-1, 1, size=(2048, 8))
    A = r.normal(size=(8, 64)) / 3.0
    T = np.sin(X @ A)
    x = torch.as_tensor(X, dtype=torch.float32, device="cuda:0")
    t = torch.as_tensor(T, dtype=torch.float32, device="cuda:0")
    losses = []
    for it in range(300):
        l = net.train_step(x, t, 3e-3)
        if it in (0, 299):
            losses.append(float(l.item()) / T.size)
    print("loss", losses, flush=True)
    assert losses[1] < 0.1 * losses[0]
    net.close()

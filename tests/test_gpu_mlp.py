"""GPU parity of the surrogate network's kernels (through the C ABI) against
the FP64 oracle.

Tolerances (FP32 on the device against FP64):
  - forward pass: max |dy| <= 2e-5 max |y|;
  - loss gradient: each layer's block within 1e-4 of the oracle's, relative to
    the block's largest entry (FP32 sums of up to 512 products);
  - Adam: the device update of every parameter within 2 % of the step size of
    the oracle update from the oracle's own gradient (Adam divides by |g|, so
    parameters with gradients near FP32 rounding move by up to lr either way),
    and the mean deviation below 0.1 % of the step size.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0911_0459_amd import lbcap
    return lbcap


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (n, 19)).astype(np.float32)
    Y = (0.5 * np.tanh(X[:, :8] @ rng.normal(0, 0.5, (8, 64)))).astype(np.float32)
    return X, Y


def _blocks():
    o, out = 0, []
    for i in range(4):
        n_in, n_out = M.DIMS[i], M.DIMS[i + 1]
        out.append((o, o + n_out * n_in))
        o += n_out * n_in
        out.append((o, o + n_out))
        o += n_out
    return out


def test_init_is_seeded_and_bounded(L):
    a, b, c = L.MLP(seed=1), L.MLP(seed=1), L.MLP(seed=2)
    assert a.param_count == M.param_count() == 153152
    pa, pb, pc = a.get_params(), b.get_params(), c.get_params()
    assert np.array_equal(pa, pb) and not np.array_equal(pa, pc)
    for (lo, hi), fan_in in zip(_blocks(), [19, 19, 256, 256, 256, 256, 256, 256]):
        blk = pa[lo:hi]
        assert np.abs(blk).max() <= 1 / np.sqrt(fan_in) + 1e-7
        assert np.abs(blk).max() > 0.9 / np.sqrt(fan_in)


@pytest.mark.parametrize("n", [1, 63, 300, 1100])
def test_forward_matches_oracle(L, n):
    net = L.MLP(seed=3)
    X, _ = _data(n, seed=n)
    y = net.predict(X)
    ref = M.forward(net.get_params().astype(np.float64), X.astype(np.float64))
    assert np.abs(y - ref).max() <= 2e-5 * np.abs(ref).max()


def test_predict_of_no_rows_is_a_no_op(L):
    net = L.MLP(seed=3)
    assert net.predict(np.zeros((0, 19), np.float32)).shape == (0, 64)


@pytest.mark.parametrize("n", [7, 512, 700])
def test_loss_gradient_matches_oracle(L, n):
    net = L.MLP(seed=4)
    X, Y = _data(n, seed=10 + n)
    loss, g = net.loss_grad(X, Y)
    loss_o, g_o = M.loss_grad(net.get_params().astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    assert abs(loss - loss_o) <= 1e-5 * loss_o
    for lo, hi in _blocks():
        scale = np.abs(g_o[lo:hi]).max()
        assert np.abs(g[lo:hi] - g_o[lo:hi]).max() <= 1e-4 * scale, (lo, hi)


def test_adam_steps_match_oracle(L):
    n, lr = 256, 1e-3
    net = L.MLP(seed=5)
    X, Y = _data(n, seed=7)
    p = net.get_params().astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 4):
        # one minibatch holding every row: the update does not depend on the shuffle
        net.train(X, Y, epochs=1, batch=n, lr=lr, seed=t)
        _, g = M.loss_grad(p, X.astype(np.float64), Y.astype(np.float64))
        p_new, m, v = M.adam_step(p, g, m, v, t, lr)
        dev = np.abs(net.get_params() - p_new)
        assert dev.max() <= 0.02 * lr * t and dev.mean() <= 1e-3 * lr
        p = net.get_params().astype(np.float64)   # follow the device trajectory


def test_training_learns_and_is_reproducible(L):
    X, Y = _data(2048, seed=11)
    a, b = L.MLP(seed=6), L.MLP(seed=6)
    l0, _ = a.loss_grad(X, Y)
    la = a.train(X, Y, epochs=60, batch=512, lr=2e-3, seed=9)
    lb = b.train(X, Y, epochs=60, batch=512, lr=2e-3, seed=9)
    assert la < 0.1 * l0
    assert la == lb and np.array_equal(a.get_params(), b.get_params())
    # short last minibatch (2048 = 3 x 600 + 248) trains as well
    c = L.MLP(seed=6)
    assert c.train(X, Y, epochs=5, batch=600, lr=2e-3, seed=9) < l0


def test_invalid_arguments_are_rejected(L):
    net = L.MLP(seed=0)
    X, Y = _data(4)
    with pytest.raises(L.LbError):
        net.train(X, Y, epochs=1, batch=0)
    with pytest.raises(L.LbError):
        net.train(X, Y, epochs=1, batch=4, lr=0.0)
    with pytest.raises(L.LbError):
        net.set_params(np.zeros(10, np.float32))

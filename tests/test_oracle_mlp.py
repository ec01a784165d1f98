"""Pins of the oracle's reference network (learned-starter extension):
gradient against central finite differences, forward pass against a
numpy evaluation written independently, and a linear special case."""
import numpy as np

P = 4801


def _params(rng, scale=0.3):
    return rng.normal(scale=scale, size=P)


def _numpy_forward(p, x):
    W1 = p[:512].reshape(64, 8)
    b1 = p[512:576]
    W2 = p[576:4672].reshape(64, 64)
    b2 = p[4672:4736]
    W3 = p[4736:4800]
    b3 = p[4800]
    a1 = np.maximum(x @ W1.T + b1, 0)
    a2 = np.maximum(a1 @ W2.T + b2, 0)
    return a2 @ W3 + b3


def test_forward_matches_numpy(oracle):
    rng = np.random.default_rng(0)
    p = _params(rng)
    x = rng.normal(size=(50, 8))
    assert np.allclose(oracle.mlp_forward(p, x), _numpy_forward(p, x), rtol=1e-13, atol=1e-13)


def test_gradient_matches_finite_differences(oracle):
    rng = np.random.default_rng(1)
    p = _params(rng)
    x = rng.normal(size=(40, 8))
    y = rng.normal(size=40)
    loss, g = oracle.mlp_loss_grad(p, x, y)
    assert abs(loss - np.mean((_numpy_forward(p, x) - y) ** 2)) < 1e-12 * (1 + loss)
    idx = np.concatenate([rng.choice(512, 20, replace=False), 512 + np.arange(5),
                          576 + rng.choice(4096, 40, replace=False), 4672 + np.arange(5),
                          4736 + rng.choice(64, 10, replace=False), [4800]])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (oracle.mlp_loss_grad(pp, x, y)[0] - oracle.mlp_loss_grad(pm, x, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * (1 + abs(g[k])), (k, fd, g[k])


def test_identity_network_special_case(oracle):
    """With W1 = [I_8; 0], positive inputs, W2 = I and W3 = e_k the network
    returns x_k exactly: pins the parameter packing."""
    p = np.zeros(P)
    W1 = np.zeros((64, 8))
    W1[:8, :8] = np.eye(8)
    p[:512] = W1.ravel()
    p[576:4672] = np.eye(64).ravel()
    for k in range(8):
        p[4736:4800] = 0
        p[4736 + k] = 1.0
        x = np.abs(np.random.default_rng(k).normal(size=(7, 8))) + 0.1
        assert np.array_equal(oracle.mlp_forward(p, x), x[:, k])

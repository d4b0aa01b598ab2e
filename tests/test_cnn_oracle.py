"""Pins of the learned-basis network oracle: library convolution, finite
differences, library Adam."""

import numpy as np
import pytest

from oracle import cnn


def test_conv_forward_matches_torch_conv3d():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 9, 9, 9))
    W = rng.normal(size=(27, 5, 4))
    b = rng.normal(size=4)
    out = cnn.conv_forward(x, W, b)
    # torch weight (co, ci, kz, ky, kx); tap = 9 (dz+1) + 3 (dy+1) + (dx+1)
    tw = torch.tensor(W.reshape(3, 3, 3, 5, 4).transpose(4, 3, 0, 1, 2).copy())
    ref = torch.nn.functional.conv3d(torch.tensor(x), tw, torch.tensor(b), padding=1).numpy()
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 9, 9, 9))
    W = rng.normal(size=(27, 3, 2))
    b = rng.normal(size=2)
    R = rng.normal(size=(2, 2, 9, 9, 9))
    gx, gW, gb = cnn.conv_backward(x, W, R)
    h = 1e-6

    def L(x_, W_, b_):
        return float((cnn.conv_forward(x_, W_, b_) * R).sum())

    for idx in [(0, 1, 4, 4, 4), (1, 2, 0, 8, 3), (0, 0, 8, 0, 0)]:
        e = np.zeros_like(x); e[idx] = h
        fd = (L(x + e, W, b) - L(x - e, W, b)) / (2 * h)
        assert abs(fd - gx[idx]) <= 1e-7 * max(1.0, abs(fd))
    for idx in [(0, 0, 0), (13, 2, 1), (26, 1, 0)]:
        e = np.zeros_like(W); e[idx] = h
        fd = (L(x, W + e, b) - L(x, W - e, b)) / (2 * h)
        assert abs(fd - gW[idx]) <= 1e-7 * max(1.0, abs(fd))
    e = np.zeros_like(b); e[1] = h
    fd = (L(x, W, b + e) - L(x, W, b - e)) / (2 * h)
    assert abs(fd - gb[1]) <= 1e-7 * max(1.0, abs(fd))


def test_network_loss_gradient_finite_differences():
    rng = np.random.default_rng(2)
    params = cnn.init_params(3)
    x = rng.normal(size=(2, 3, 9, 9, 9))
    target = rng.dirichlet(np.ones(8), size=(2, 7, 7, 7)).transpose(0, 4, 1, 2, 3)
    loss, g = cnn.loss_and_grad(params, x, target)
    h = 1e-6
    o = 0
    offsets = []
    for ci, co in cnn.LAYERS:
        offsets.append(o)
        o += 27 * ci * co + co
    for li, off in enumerate(offsets):
        for j in (0, 7, 27 * cnn.LAYERS[li][0] * cnn.LAYERS[li][1] + 1):   # two weights and a bias
            k = off + j
            e = np.zeros_like(params); e[k] = h
            lp, _ = cnn.loss_and_grad(params + e, x, target)
            lm, _ = cnn.loss_and_grad(params - e, x, target)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k]) <= 1e-7 * max(abs(fd), 1e-6) + 1e-11, (li, j, fd, g[k])


def test_softmax_is_a_partition_of_unity():
    rng = np.random.default_rng(4)
    phi, _ = cnn.forward(cnn.init_params(5), rng.normal(size=(1, 3, 9, 9, 9)))
    assert np.allclose(phi.sum(axis=1), 1.0, atol=1e-14) and phi.min() >= 0


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(3)]
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = cnn.adam_step(p, g, m, v, t, lr=1e-2)
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_loss_window_hand_worked():
    """The loss compares the network output on the 7x7x7 interior cells of the
    9x9x9 patch (patch positions 1..7 on each axis) with the targets, in the
    same (z, y, x) order.  Hand-worked case: a network that passes input
    channel 0 through every layer at the centre tap to output channel 0
    (all other weights and biases 0) gives logits z_0 = x_0, z_1..7 = 0, so
    phi = (e^x0, 1, ..., 1) / (e^x0 + 7).  With x_0 = ln 7 at patch cell
    (z, y, x) = (7, 1, 1) and at (8, 8, 8) (a vertex plane, outside the
    interior), 0 elsewhere, phi is uniform 1/8 except phi = (1/2, 1/14, ...)
    at those two cells.  Targets: uniform 1/8, except interior index
    (6, 0, 0) (= patch cell (7, 1, 1)) set to (1/2, 1/14, ...) and interior
    index (0, 0, 0) set to the same vector.  Only interior (0, 0, 0) then
    differs: (1/2 - 1/8)^2 + 7 (1/14 - 1/8)^2 = 9/56, so the loss is
    9 / (56 * 8 * 343).  A window shifted by one cell, a transposed window
    or a loss over all 9^3 cells gives another value."""
    params = np.zeros(cnn.num_params())
    o = 0
    for li, (ci, co) in enumerate(cnn.LAYERS):
        W = np.zeros((27, ci, co))
        W[13, 0, 0] = 1.0          # centre tap, channel 0 -> channel 0
        params[o:o + W.size] = W.ravel()
        o += W.size + co            # biases stay 0
    x = np.zeros((1, 3, 9, 9, 9))
    x[0, 0, 7, 1, 1] = np.log(7.0)
    x[0, 0, 8, 8, 8] = np.log(7.0)
    hot = np.array([0.5] + [1.0 / 14.0] * 7)
    target = np.full((1, 8, 7, 7, 7), 1.0 / 8.0)
    target[0, :, 6, 0, 0] = hot
    target[0, :, 0, 0, 0] = hot
    phi, _ = cnn.forward(params, x)
    assert np.allclose(phi[0, :, 7, 1, 1], hot, rtol=1e-14) and np.allclose(phi[0, :, 8, 8, 8], hot, rtol=1e-14)
    loss, _ = cnn.loss_and_grad(params, x, target)
    assert abs(loss - 9.0 / (56.0 * 8 * 343)) <= 1e-15

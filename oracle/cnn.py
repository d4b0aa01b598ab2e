"""CPU oracle of the learned-basis network — TEST INFRASTRUCTURE ONLY.

Plain FP64 NumPy: 3D convolution with 3x3x3 kernels and zero "same"
padding, ReLU, softmax over the 8 vertex channels, mean-squared error on the
interior cells of a 9x9x9 dual-block patch, and the Adam update.  Forward and
backward are written per kernel tap (27 shifted copies), no im2col or FFT.

Conventions (shared with the GPU kernels as specification, not code):
  activations x[b, c, z, y, x] for one 9x9x9 patch per batch entry;
  weights W[tap, ci, co] with tap = 9 (dz+1) + 3 (dy+1) + (dx+1);
  output[b, co, p] = bias[co] + sum_{tap, ci} W[tap, ci, co] x[b, ci, p + d(tap)]
  (a cross-correlation; neighbours outside the patch read zero).
Network: conv(3->32) ReLU, conv(32->32) ReLU, conv(32->32) ReLU, conv(32->8),
softmax over the 8 channels, loss on the 7x7x7 interior cells.

Parity status: pinned by finite differences (central, h = 1e-6) and by
torch.nn.functional.conv3d / torch.optim.Adam on the CPU.
"""

from __future__ import annotations

import numpy as np

LAYERS = [(3, 32), (32, 32), (32, 32), (32, 8)]
D = 9


def taps():
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                out.append((dz, dy, dx))
    return out


def _shift(x, dz, dy, dx):
    """y[..., z, y, x] = x[..., z+dz, y+dy, x+dx], zero outside."""
    out = np.zeros_like(x)
    Dz, Dy, Dx = x.shape[-3:]
    zs, ze = max(0, -dz), min(Dz, Dz - dz)
    ys, ye = max(0, -dy), min(Dy, Dy - dy)
    xs, xe = max(0, -dx), min(Dx, Dx - dx)
    out[..., zs:ze, ys:ye, xs:xe] = x[..., zs + dz:ze + dz, ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv_forward(x, W, b):
    """x: (B, Ci, 9, 9, 9), W: (27, Ci, Co), b: (Co,) -> (B, Co, 9, 9, 9)."""
    B = x.shape[0]
    Co = W.shape[2]
    out = np.zeros((B, Co) + x.shape[2:])
    for t, (dz, dy, dx) in enumerate(taps()):
        xs = _shift(x, dz, dy, dx)
        out += np.einsum("bizyx,io->bozyx", xs, W[t])
    return out + b[None, :, None, None, None]


def conv_backward(x, W, gout):
    """Gradients of sum(gout * conv_forward(x, W, b)) wrt x, W and b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(taps()):
        xs = _shift(x, dz, dy, dx)
        gW[t] = np.einsum("bizyx,bozyx->io", xs, gout)
        # d/dx of x[p + d] * g[p]: g shifted back by -d
        gx += _shift(np.einsum("bozyx,io->bizyx", gout, W[t]), -dz, -dy, -dx)
    gb = gout.sum(axis=(0, 2, 3, 4))
    return gx, gW, gb


def softmax(z):
    """Softmax over axis 1 (the 8 vertex channels)."""
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=1, keepdims=True)


def interior_mask():
    m = np.zeros((D, D, D), dtype=bool)
    m[1:-1, 1:-1, 1:-1] = True
    return m


def unpack(params):
    """Flat parameter vector -> [(W, b)] per layer (W: (27, Ci, Co))."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = params[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        b = params[o:o + co]
        o += co
        out.append((W, b))
    assert o == params.size
    return out


def num_params():
    return sum(27 * ci * co + co for ci, co in LAYERS)


def init_params(seed):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=27 * ci * co))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def forward(params, x):
    """Returns (phi (B, 8, 9, 9, 9), cache)."""
    layers = unpack(params)
    acts = [x]
    h = x
    for li, (W, b) in enumerate(layers):
        z = conv_forward(h, W, b)
        if li < len(layers) - 1:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    phi = softmax(h)
    return phi, (acts, h)


def loss_and_grad(params, x, target):
    """MSE over the interior cells and 8 channels; target (B, 8, 7, 7, 7).
    Returns (loss, grad (flat))."""
    layers = unpack(params)
    phi, (acts, logits) = forward(params, x)
    m = interior_mask()
    B = x.shape[0]
    nterm = B * 8 * m.sum()
    diff = np.zeros_like(phi)
    diff[:, :, 1:-1, 1:-1, 1:-1] = phi[:, :, 1:-1, 1:-1, 1:-1] - target
    loss = float((diff ** 2).sum() / nterm)
    gphi = 2.0 * diff / nterm
    # softmax backward: g_z = phi * (g_phi - sum_c phi_c g_phi_c)
    g = phi * (gphi - (phi * gphi).sum(axis=1, keepdims=True))
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        gx, gW, gb = conv_backward(acts[li], W, g)
        grads[li] = (gW, gb)
        if li > 0:
            g = gx * (acts[li] > 0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v

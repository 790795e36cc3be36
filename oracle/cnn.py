"""CPU reference of the learned warm-start network (test infrastructure).

Plain FP64 numpy: four 3x3 convolutions with zero ("same") padding,
7 -> 32 -> 32 -> 32 -> 3 channels, exact-erf GELU after the first three,
mean-squared-error loss, backward pass by the chain rule, and the Adam
update.  With bf16=True the inputs, weights and stored activations are
rounded to bfloat16 (round to nearest even) at the points where the GPU
kernels store bfloat16, and accumulation stays in high precision, so the
GPU (FP32 accumulate) can be compared at the bfloat16 level.

Parameter vector layout (shared with the library's documented ABI): for
each layer l, W_l[co][ci][3][3] followed by b_l[co].
"""
import math

import numpy as np
from scipy.special import erf

LAYERS = [(7, 32), (32, 32), (32, 32), (32, 3)]


def param_count():
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def unpack(params):
    out, off = [], 0
    for ci, co in LAYERS:
        W = params[off: off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = params[off: off + co]
        off += co
        out.append((W, b))
    return out


def to_bf16(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def conv3x3(x, W, b):
    """y[b,co,i,j] = b[co] + sum_{ci,di,dj} W[co,ci,di,dj] x[b,ci,i+di-1,j+dj-1] (zeros outside)."""
    B, C, H, Wd = x.shape
    xp = np.zeros((B, C, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, W.shape[0], H, Wd))
    for di in range(3):
        for dj in range(3):
            y += np.einsum("oc,bchw->bohw", W[:, :, di, dj], xp[:, :, di:di + H, dj:dj + Wd])
    return y + b[None, :, None, None]


def conv3x3_backward(x, W, dy):
    """Gradients of conv3x3 with respect to W, b and x."""
    B, C, H, Wd = x.shape
    xp = np.zeros((B, C, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for di in range(3):
        for dj in range(3):
            dW[:, :, di, dj] = np.einsum("bohw,bchw->oc", dy, xp[:, :, di:di + H, dj:dj + Wd])
            dxp[:, :, di:di + H, dj:dj + Wd] += np.einsum("oc,bohw->bchw", W[:, :, di, dj], dy)
    db = dy.sum(axis=(0, 2, 3))
    return dW, db, dxp[:, :, 1:-1, 1:-1]


def forward(params, x, bf16=False, keep=False):
    layers = unpack(params)
    r = to_bf16 if bf16 else (lambda v: v)
    a = r(x)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = conv3x3(a, r(W), b)  # biases stay FP32 on the GPU
        cache.append((a, z))
        if l < 3:
            a = r(gelu(z))
        else:
            a = z
    return (a, cache) if keep else a


def loss_and_grad(params, x, target, bf16=False):
    """MSE over every output element and its gradient (same layout as params)."""
    layers = unpack(params)
    r = to_bf16 if bf16 else (lambda v: v)
    out, cache = forward(params, x, bf16=bf16, keep=True)
    n = out.size
    loss = float(((out - target) ** 2).sum() / n)
    dz = 2.0 * (out - target) / n
    grads = [None] * 4
    for l in range(3, -1, -1):
        a_prev, z = cache[l]
        W, b = layers[l]
        if bf16:
            dz = r(dz)
        dW, db, da = conv3x3_backward(a_prev, r(W), dz)
        grads[l] = (dW, db)
        if l > 0:
            dz = da * gelu_grad(cache[l - 1][1])
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()]) for g in grads])
    return loss, flat


def adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), in place on params, m and v."""
    m[:] = b1 * m + (1 - b1) * grad
    v[:] = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    params -= lr * mh / (np.sqrt(vh) + eps)

"""FP64 oracle of the learned warm start's network and of its matrix-core GEMM.

TEST INFRASTRUCTURE ONLY (same rules as the rest of this package): only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg
use it; the GPU path never imports it.

The network maps theta to  o = W3 h2 + b3,  h2 = relu(W2 h1 + b2),
h1 = relu(W1 theta + b1), with the loss  L = sum (o - t)^2 / (2 B out)  over a
batch of B rows.  Its gradient is written out by the chain rule (plain
backpropagation).  ``quantize=True`` places a BF16 rounding (round to nearest,
ties to even, from the FP32 value) at every GEMM operand, as the GPU path
does, and evaluates every product and sum in FP64; ``quantize=False`` is the
exact network, the one the finite-difference tests pin.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest BF16 (ties to even) through FP32; returns float64.
    A BF16 number is an FP32 number whose low 16 bits are zero."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def unpack(p, n_in, hid, n_out):
    """Flat parameter vector -> (W1 [hid x in], b1, W2 [hid x hid], b2, W3 [out x hid], b3)."""
    p = np.asarray(p, dtype=np.float64)
    sizes = [hid * n_in, hid, hid * hid, hid, n_out * hid, n_out]
    parts, o = [], 0
    for s in sizes:
        parts.append(p[o:o + s])
        o += s
    W1, b1, W2, b2, W3, b3 = parts
    return W1.reshape(hid, n_in), b1, W2.reshape(hid, hid), b2, W3.reshape(n_out, hid), b3


def forward(p, theta, n_in, hid, n_out, quantize=True):
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, hid, n_out)
    x = q(theta)
    h1 = np.maximum(x @ q(W1).T + b1, 0.0)
    h1 = f32(h1) if quantize else h1
    h2 = np.maximum(q(h1) @ q(W2).T + b2, 0.0)
    h2 = f32(h2) if quantize else h2
    o = q(h2) @ q(W3).T + b3
    return {"x": x, "h1": h1, "h2": h2, "o": o}


def loss_and_grad(p, theta, target, n_in, hid, n_out, quantize=True):
    """(L, flat gradient) of L = sum (o - target)^2 / (2 B n_out)."""
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, hid, n_out)
    f = forward(p, theta, n_in, hid, n_out, quantize)
    B = theta.shape[0]
    r = f["o"] - np.asarray(target, dtype=np.float64)
    loss = float((r * r).sum() / (2.0 * B * n_out))
    d_o = r / (B * n_out)
    if quantize:
        d_o = f32(d_o)
    gW3 = q(d_o).T @ q(f["h2"])
    gb3 = d_o.sum(axis=0)
    dh2 = q(d_o) @ q(W3)
    dz2 = np.where(f["h2"] > 0.0, dh2, 0.0)
    dz2 = f32(dz2) if quantize else dz2
    gW2 = q(dz2).T @ q(f["h1"])
    gb2 = dz2.sum(axis=0)
    dh1 = q(dz2) @ q(W2)
    dz1 = np.where(f["h1"] > 0.0, dh1, 0.0)
    dz1 = f32(dz1) if quantize else dz1
    gW1 = q(dz1).T @ f["x"]
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def gemm(a, b, ta=0, tb=0, bias=None, relu=False):
    """C = op(A) op(B) (+ bias) (relu) of BF16 operands (given as float values),
    in FP64, and the bound |C_gpu - C| <= K 2^-24 sum_k |op(A)_mk op(B)_kn| of a
    product formed with exact products and FP32 sums."""
    A = np.asarray(a, dtype=np.float64)
    Bm = np.asarray(b, dtype=np.float64)
    A = A.T if ta else A
    Bm = Bm.T if tb else Bm
    c = A @ Bm
    absum = np.abs(A) @ np.abs(Bm)
    K = A.shape[1]
    bound = K * 2.0 ** -24 * absum
    if bias is not None:
        c = c + np.asarray(bias, dtype=np.float64)
        bound = bound + 2.0 ** -24 * np.abs(c)
    if relu:
        c = np.maximum(c, 0.0)
    return c, bound

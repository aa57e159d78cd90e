"""FP64 reference of the learned amplitude-update network (test infrastructure).

The paper has no learned component; this is the reference for the library's own network:
inputs x (n_in features per amplitude) -> h1 = tanh(W1 x + b1) -> h2 = tanh(W2 h1 + b2) ->
y = W3 h2 + b3, y = (Re g, Im g).  For a sample with Jacobi step q (the step the gain
multiplies) and target correction r = (t* - t) - q, the loss of a minibatch is
    loss = sum_s |r_s - q_s g_s|^2 / sum_s |q_s|^2 .
Parameters are one flat vector in the order W1 (n_h x n_in, row-major), b1, W2 (n_h x n_h), b2,
W3 (n_out x n_h), b3.  Gradients here come from central finite differences of `loss`, so they
are independent of any backpropagation code.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 4, 64, 2


def sizes(n_in=N_IN, n_h=N_H, n_out=N_OUT):
    return [n_h * n_in, n_h, n_h * n_h, n_h, n_out * n_h, n_out]


def unpack(p, n_in=N_IN, n_h=N_H, n_out=N_OUT):
    out, o = [], 0
    shapes = [(n_h, n_in), (n_h,), (n_h, n_h), (n_h,), (n_out, n_h), (n_out,)]
    for s in shapes:
        k = int(np.prod(s))
        out.append(np.asarray(p[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def round_bf16(x):
    """Nearest BF16 value (ties to even) of each entry, through its FP32 value."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X, h1_bf16=False):
    """y = W3 tanh(W2 h1 + b2) + b3 with h1 = tanh(W1 x + b1); h1_bf16 stores h1 in BF16 first (the
    precision of the solver's inference, whose hidden product runs on BF16 matrix cores)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = np.tanh(X @ W1.T + b1)
    if h1_bf16:
        h1 = round_bf16(h1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3


def loss(p, X, q, r):
    """q, r: complex arrays of the minibatch."""
    y = forward(p, np.asarray(X, dtype=np.float64))
    g = y[:, 0] + 1j * y[:, 1]
    e = r - q * g
    return float(np.sum(np.abs(e) ** 2) / np.sum(np.abs(q) ** 2))


def fd_grad(p, X, q, r, h=1e-6, idx=None):
    """Central finite-difference gradient of `loss` (all parameters or the indices `idx`)."""
    p = np.asarray(p, dtype=np.float64)
    idx = range(p.size) if idx is None else idx
    out = {}
    for k in idx:
        a, b = p.copy(), p.copy()
        a[k] += h
        b[k] -= h
        out[k] = (loss(a, X, q, r) - loss(b, X, q, r)) / (2 * h)
    return out

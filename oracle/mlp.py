"""The coefficient network in FP64: forward, backward, Adam (test infrastructure only).

Architecture (reading of "3 layers of width 64"): inputs x in R^6 standardised
as z = (x - mean) / std, three tanh hidden layers of width 64, linear output in
R^8:
    h1 = tanh(W1 z + b1), h2 = tanh(W2 h1 + b2), h3 = tanh(W3 h2 + b3),
    y = W4 h3 + b4,
with W shaped (out, in).  The coefficients of the learned step are
c = c_Euler(h) + y.

Loss over a batch of S samples with defect data (G_s, b_s, f_s):
    L = (1/S) sum_s [(c_s^T G_s c_s - 2 b_s^T c_s + f_s) / f_s + rho |c_s,q|^2],
    dL/dc_s = [2 (G_s c_s - b_s) / f_s + 2 rho D_q c_s] / S,
with c_s,q = (c4, .., c7) and D_q the matching 0/1 diagonal (rho = 1e-6).

Adam: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
      p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parity: backward pinned by central finite differences of the forward loss
(tests/test_oracle_mlp.py); forward is the plain definition above.
"""

import numpy as np

SIZES = (6, 64, 64, 64, 8)


def n_params():
    return sum(o * i + o for i, o in zip(SIZES[:-1], SIZES[1:]))


def unflatten(theta):
    """Flat parameter vector -> [(W1, b1), ..., (W4, b4)].

    Flat layout, layer by layer: W (out x in, row-major) then b.
    """
    out = []
    off = 0
    for i, o in zip(SIZES[:-1], SIZES[1:]):
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def forward(theta, Z):
    """Z: (S, 6) standardised inputs.  Returns (Y (S, 8), cache)."""
    layers = unflatten(theta)
    acts = [Z]
    H = Z
    for li, (W, b) in enumerate(layers):
        pre = H @ W.T + b
        H = np.tanh(pre) if li < len(layers) - 1 else pre
        acts.append(H)
    return H, acts


def backward(theta, acts, dY):
    """Gradient of a scalar loss wrt theta given dL/dY (S, 8)."""
    layers = unflatten(theta)
    grads = []
    d = dY
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        H_in = acts[li]
        gW = d.T @ H_in
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            d = (d @ W) * (1.0 - acts[li] ** 2)
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


RHO = 1e-6
DQ = np.array([0.0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 1.0])


def loss_and_grad_y(Y, c_base, G, b, f, rho=RHO):
    """Loss over the batch and dL/dY.  c = c_base + Y; shapes (S,8),(S,8),(S,8,8),(S,8),(S,)."""
    C = c_base + Y
    GC = np.einsum("sab,sb->sa", G, C)
    per = (np.einsum("sa,sa->s", C, GC) - 2 * np.einsum("sa,sa->s", b, C) + f) / f
    per = per + rho * np.sum(DQ * C * C, axis=1)
    S = Y.shape[0]
    dY = (2.0 * (GC - b) / f[:, None] + 2.0 * rho * DQ * C) / S
    return float(per.mean()), dY


def loss(theta, Z, c_base, G, b, f, rho=RHO):
    Y, _ = forward(theta, Z)
    return loss_and_grad_y(Y, c_base, G, b, f, rho)[0]


def loss_grad(theta, Z, c_base, G, b, f, rho=RHO):
    Y, acts = forward(theta, Z)
    L, dY = loss_and_grad_y(Y, c_base, G, b, f, rho)
    return L, backward(theta, acts, dY)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step count).  Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v

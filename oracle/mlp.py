"""Oracle of the learned starting guess for the inverse iteration.

TEST INFRASTRUCTURE ONLY (used by the test-suite to check the GPU kernels).

A two-layer perceptron y = W2 tanh(W1 d + b1) + b2 with hidden width 128 maps
an atom-pair block descriptor d = [(r_i - r_j)/R, |r_i - r_j|/R, S_ij] to a
correction of the first-order start 2 delta_ij I - S_ij of the inverse
(the iteration itself is Sec. V.A's Hotelling method).  Plain numpy FP64; the
forward pass uses W1 and W2 rounded to FP16, as the GPU does, and the
gradients are those of the loss at the rounded weights.
"""

import numpy as np

HIDDEN = 128


def split(w, n_in, n_out, h=HIDDEN):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + h * n_in].reshape(h, n_in); o += h * n_in
    b1 = w[o:o + h]; o += h
    W2 = w[o:o + n_out * h].reshape(n_out, h); o += n_out * h
    b2 = w[o:o + n_out]; o += n_out
    assert o == w.size
    return W1, b1, W2, b2


def n_params(n_in, n_out, h=HIDDEN):
    return h * n_in + h + n_out * h + n_out


def forward(w, x, n_in, n_out, fp16=True):
    W1, b1, W2, b2 = split(w, n_in, n_out)
    if fp16:
        W1 = W1.astype(np.float16).astype(np.float64)
        W2 = W2.astype(np.float16).astype(np.float64)
    h = np.tanh(np.asarray(x, np.float64) @ W1.T + b1)
    return h @ W2.T + b2, h


def loss_grad(w, x, t, n_in, n_out, fp16=True):
    """Mean squared error per output element and its gradient (flat, like w)."""
    x = np.asarray(x, np.float64)
    t = np.asarray(t, np.float64)
    W1, b1, W2, b2 = split(w, n_in, n_out)
    if fp16:
        W2 = W2.astype(np.float16).astype(np.float64)
    y, h = forward(w, x, n_in, n_out, fp16)
    n = x.shape[0]
    d = y - t
    loss = float((d * d).sum() / (n * n_out))
    dy = 2.0 * d / (n * n_out)
    dW2 = dy.T @ h
    db2 = dy.sum(axis=0)
    dh = (dy @ W2) * (1.0 - h * h)
    dW1 = dh.T @ x
    db1 = dh.sum(axis=0)
    return loss, np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2])


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Step t (1, 2, ...) of Adam (Kingma and Ba, 2015, Algorithm 1): the
    moments m <- beta1 m + (1 - beta1) g and v <- beta2 v + (1 - beta2) g^2,
    their bias-corrected values m / (1 - beta1^t) and v / (1 - beta2^t), and
    w <- w - lr m_hat / (sqrt(v_hat) + eps).  Returns (w, m, v)."""
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return np.asarray(w, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def descriptors(xyz, S, R):
    """d for every block of S (oracle BSM on S's pattern), in S's block order."""
    r = S.pat.rows()
    c = S.pat.col.astype(np.int64)
    dv = xyz[r] - xyz[c]
    dist = np.sqrt((dv * dv).sum(axis=1))
    return np.concatenate([dv / R, dist[:, None] / R, S.val.real.reshape(S.val.shape[0], -1)], axis=1)


def first_order_start(S):
    """Blocks of 2 delta_ij I - S_ij on S's pattern (real)."""
    b = S.b
    out = -S.val.real.copy()
    d = S.pat.index(np.arange(S.pat.n), np.arange(S.pat.n))
    out[d] += 2.0 * np.eye(b)
    return out

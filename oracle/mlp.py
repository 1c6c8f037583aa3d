"""FP64 reference of the small MLP that predicts initial multicanonical
weights -- TEST INFRASTRUCTURE ONLY.

Network: x (2) -> tanh(W1 x + b1) (64) -> tanh(W2 h1 + b2) (64) -> W3 h2 + b3
(1); 4417 parameters, flattened in the order W1 [64][2], b1 [64], W2 [64][64],
b2 [64], W3 [1][64], b3 [1].  Loss: mean squared error over the data set.
Optimiser: Adam (bias-corrected moments).  Initialisation: Xavier-uniform
weights w = (2u - 1) sqrt(6 / (fan_in + fan_out)), u = (r >> 8) 2^-24 with r
the Philox word of parameter index idx (tag MLP_INIT, counter idx / 4, word
idx mod 4), biases zero.  Inputs are (E/N + 1, 32/L - 1); the target is the
entropy deficit -ln W(E) / N with ln W(0) = 0, less an analytic baseline (the
entropy of independent flipped spins) that carries its ground-state
singularity.

The backward pass is the chain rule written out; the tests pin it against
central finite differences of the loss.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

H = 64
SHAPES = [("W1", (H, 2)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (1, H)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 4417


def unflatten(p):
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[off:off + n].reshape(shape)
        off += n
    return out


def init_params(seed):
    """Xavier-uniform weights from the Philox stream, zero biases (float64
    values of the float32 parameters)."""
    p = np.zeros(NPARAMS, dtype=np.float64)
    off = 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        if name.startswith("W"):
            fan_out, fan_in = shape
            a = math.sqrt(6.0 / (fan_in + fan_out))
            for i in range(n):
                r = oracle.draw_word(seed, oracle.TAG_MLP_INIT, off + i, 0, 0)
                u = (r >> 8) * (1.0 / 16777216.0)
                p[off + i] = float(np.float32((2.0 * u - 1.0) * a))
        off += n
    return p


def features(E, N, L):
    """Network inputs for energies E of an L x L lattice with N sites."""
    E = np.asarray(E, dtype=np.float64)
    return np.stack([E / N + 1.0, np.full_like(E, 32.0 / L - 1.0)], axis=1)


def forward(p, X):
    q = unflatten(p)
    z1 = X @ q["W1"].T + q["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.tanh(z2)
    y = h2 @ q["W3"].T + q["b3"]
    return y[:, 0], (h1, h2)


def loss_and_grad(p, X, Y):
    """MSE loss and its gradient by the chain rule."""
    q = unflatten(p)
    n = X.shape[0]
    y, (h1, h2) = forward(p, X)
    r = y - Y
    loss = float(np.mean(r * r))
    dy = (2.0 / n) * r[:, None]              # dL/dy, [n, 1]
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dz2 = (dy @ q["W3"]) * (1.0 - h2 * h2)   # [n, 64]
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ q["W2"]) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return loss, np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])


def train(p, X, Y, epochs, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Full-batch Adam; returns the parameters and the loss before each step."""
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for t in range(1, epochs + 1):
        loss, g = loss_and_grad(p, X, Y)
        losses.append(loss)
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        p = p - lr * mh / (np.sqrt(vh) + eps)
    return p, np.array(losses)


def _gas_entropy(x):
    """Entropy per site of independent flipped spins at density x: -x ln x -
    (1 - x) ln(1 - x), 0 at x = 0 (libm log and log1p, as the library)."""
    return 0.0 if x <= 0.0 else -x * math.log(x) - (1.0 - x) * math.log1p(-x)


def baseline(L):
    """Output baseline b(k) = h(k / 2N) - h(1/4), h the entropy of a gas of
    independent flipped spins (the low-energy behaviour of g(E), where a site
    in the window's lower end has an isolated flipped spin per 8 of energy),
    so that the network fits the smooth remainder instead of the x ln x
    singularity at the ground state."""
    N = L * L
    K = N // 2
    b = np.array([_gas_entropy(k / (2.0 * N)) for k in range(K + 1)])
    return b - b[K]


def training_set(lnW_by_L):
    """(X, Y) from converged ln W per L: every window level but k = 1, with
    ln W taken relative to its value at E = 0 (level N/2), minus the
    baseline: y = -(ln W - ln W(0)) / N - b."""
    X, Y = [], []
    for L, lnW in sorted(lnW_by_L.items()):
        N = L * L
        K = N // 2
        lnW = np.asarray(lnW, dtype=np.float64)
        b = baseline(L)
        k = np.array([i for i in range(K + 1) if i != 1])
        E = 4 * k - 2 * N
        X.append(features(E, N, L))
        Y.append(-(lnW[k] - lnW[K]) / N - b[k])
    return np.concatenate(X), np.concatenate(Y)


def predict_lnW(p, L):
    """Initial ln W(E) = -N (y(E/N, 1/L) + b) over the window levels, shifted
    to ln W(0) = 0."""
    N = L * L
    K = N // 2
    E = 4 * np.arange(K + 1) - 2 * N
    y, _ = forward(p, features(E, N, L))
    lnW = -N * (y + baseline(L))
    return lnW - lnW[K]

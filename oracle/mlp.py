"""Plain FP64 oracle of the warm-start network (test infrastructure).

A fully connected network x -> SiLU(x W1 + b1) -> SiLU(. W2 + b2) ->
SiLU(. W3 + b3) -> . W4 + b4 that predicts the Newton increment of the
reduced coordinates of a load step from per-point features; silu(z) = z
sigmoid(z).  Loss: mean over the batch of the summed squared error.  Forward,
backward (hand-derived chain rule) and one Adam update (Kingma & Ba 2015,
with bias correction), written out plainly so that the GPU kernels can be
compared with them.  Weights W_l are stored (fan_in, fan_out), row-major.
"""
import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init(dims, seed):
    """He-uniform style initialisation from a seeded generator."""
    g = np.random.Generator(np.random.PCG64(seed))
    params = []
    for fi, fo in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / fi) * (0.5 if fo == dims[-1] else 1.0)
        params.append(g.uniform(-lim, lim, size=(fi, fo)))
        params.append(np.zeros(fo))
    return params


def bf16(x):
    """Round to the nearest bfloat16 (8 significand bits, ties to even), via
    the nearest float32: the top 16 bits of the float32 pattern after adding
    0x7fff plus the lowest kept bit.  Returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, X, bf16_operands=False):
    """Returns output and the cache (pre-activations, activations).  With
    bf16_operands every product takes its two operands rounded to bfloat16
    (activations and weights), the sums exact; the biases, the SiLU and the
    cached activations stay unrounded."""
    a = X
    zs, acts = [], [X]
    L = len(params) // 2
    for l in range(L):
        W, b = params[2 * l], params[2 * l + 1]
        z = (bf16(a) @ bf16(W) if bf16_operands else a @ W) + b
        zs.append(z)
        a = silu(z) if l < L - 1 else z
        acts.append(a)
    return a, (zs, acts)


def loss(params, X, Y):
    out, _ = forward(params, X)
    return float(np.mean(np.sum((out - Y) ** 2, axis=1)))


def backward(params, X, Y, bf16_operands=False):
    """Loss and gradients (same order as params); the forward pass as in
    forward(), the backward pass unrounded."""
    out, (zs, acts) = forward(params, X, bf16_operands)
    B = X.shape[0]
    L = len(params) // 2
    grads = [None] * len(params)
    d = 2.0 * (out - Y) / B  # dLoss/dout
    for l in reversed(range(L)):
        if l < L - 1:
            d = d * dsilu(zs[l])
        grads[2 * l] = acts[l].T @ d
        grads[2 * l + 1] = d.sum(axis=0)
        d = d @ params[2 * l].T
    return float(np.mean(np.sum((out - Y) ** 2, axis=1))), grads


def adam(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t starts at 1); returns new params, m, v."""
    newp, newm, newv = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1 - beta1) * g
        vi = beta2 * vi + (1 - beta2) * g * g
        mh = mi / (1 - beta1 ** t)
        vh = vi / (1 - beta2 ** t)
        newp.append(p - lr * mh / (np.sqrt(vh) + eps))
        newm.append(mi)
        newv.append(vi)
    return newp, newm, newv


def plastic_statistics(wJ, hist):
    """Eight summary statistics of the committed plastic state of one point.

    wJ: (m,) ECM weight times |det F_mu|; hist = (Fp (m,2,2), Fp33 (m,), xi (m,)).
    Returns [weighted mean xi, max xi, weighted std xi, weighted fraction with
    xi > 0, weighted mean of (F^pl - I) in-plane (4 entries)].
    """
    Fp, Fp33, xi = hist
    w = wJ / wJ.sum()
    mean = float(w @ xi)
    std = float(np.sqrt(max(w @ (xi - mean) ** 2, 0.0)))
    frac = float(w @ (xi > 0))
    dFp = (Fp - np.eye(2)).reshape(-1, 4)
    return np.concatenate([[mean, float(xi.max()), std, frac], w @ dFp])

"""Pins of the warm-start network oracle: hand-derived gradients against
central finite differences, the first Adam step in closed form, and the
plastic summary statistics on a hand-made state."""
import numpy as np

from oracle import mlp

DIMS = [54, 16, 16, 16, 40]


def test_gradients_match_finite_differences():
    params = mlp.init(DIMS, 0)
    g = np.random.Generator(np.random.PCG64(1))
    X = g.normal(size=(7, DIMS[0]))
    Y = g.normal(size=(7, DIMS[-1]))
    L0, grads = mlp.backward(params, X, Y)
    assert abs(L0 - mlp.loss(params, X, Y)) < 1e-14
    h = 1e-6
    for pi in range(len(params)):
        flat = params[pi].reshape(-1)
        idx = g.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            Lp = mlp.loss(params, X, Y)
            flat[i] = old - h
            Lm = mlp.loss(params, X, Y)
            flat[i] = old
            fd = (Lp - Lm) / (2 * h)
            an = grads[pi].reshape(-1)[i]
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (pi, i, fd, an)


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.abs(mlp.dsilu(z) - (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)).max() < 1e-9


def test_first_adam_step_closed_form():
    # with bias correction the first step is lr * g / (|g| + eps)
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    z = [np.zeros(3)]
    newp, m, v = mlp.adam(p, g, z, z, 1, 0.01)
    expect = p[0] - 0.01 * g[0] / (np.abs(g[0]) + 1e-8)
    assert np.abs(newp[0] - expect).max() < 1e-15


def test_plastic_statistics_by_hand():
    wJ = np.array([1.0, 3.0])
    Fp = np.stack([np.eye(2), np.array([[1.1, 0.2], [0.0, 0.9]])])
    xi = np.array([0.0, 0.2])
    s = mlp.plastic_statistics(wJ, (Fp, np.ones(2), xi))
    assert np.allclose(s, [0.15, 0.2, np.sqrt(0.25 * 0.15 ** 2 + 0.75 * 0.05 ** 2), 0.75,
                           0.075, 0.15, 0.0, -0.075], atol=1e-15)


def test_bf16_rounding_and_forward():
    """bfloat16 keeps 8 significand bits: 1 + 2^-7 is exact, 1 + 2^-8 is a tie
    going to the even 1, 1 + 3 * 2^-8 a tie going up to 1 + 2^-6, 1 + 2^-8 +
    2^-20 rounds up (truncation would not); sign and exponent are kept.  With
    weights and inputs that are bfloat16 numbers already, the first layer's
    pre-activations are the same with and without rounded operands; deeper
    layers differ only by the rounding of the hidden activations."""
    x = np.array([1.0, 1 + 2 ** -7, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -3.0, 2.0 ** -130])
    r = mlp.bf16(x)
    assert np.array_equal(r[:6], [1.0, 1 + 2 ** -7, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -3.0])
    assert r[6] == 2.0 ** -130  # subnormal in float32, a single significant bit
    g = np.random.Generator(np.random.PCG64(5))
    params = [mlp.bf16(p) for p in mlp.init([6, 5, 5, 5, 3], 2)]
    X = mlp.bf16(g.normal(size=(4, 6)))
    a, _ = mlp.forward(params, X)
    b, (zs, _) = mlp.forward(params, X, bf16_operands=True)
    z0 = X @ params[0] + params[1]
    assert np.array_equal(zs[0], z0)  # first layer: the operands are bfloat16 already
    assert np.abs(a - b).max() < 2e-2 * np.abs(a).max() and not np.array_equal(a, b)

"""Pins of the FP64 warm-start network reference against the mathematics."""
import math

import numpy as np

from oracle import mlp
import workloads as W


def test_bf16_rounding_known_patterns():
    # BF16 keeps 7 mantissa bits: the spacing at 1 is 2^-7
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0                       # tie, even mantissa kept
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6        # tie, rounds up to even
    assert mlp.bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7  # above the tie
    assert mlp.bf16(-3.0) == -3.0
    assert mlp.bf16(2.0 ** -130) > 0.0                             # FP32 subnormal survives


def test_gelu_special_values():
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15   # Phi(1) of the standard normal
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-12 and abs(mlp.gelu(-10.0)) < 1e-12
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-15
    z = np.linspace(-4, 4, 41)
    fd = (mlp.gelu(z + 1e-6) - mlp.gelu(z - 1e-6)) / 2e-6
    assert np.abs(fd - mlp.gelu_grad(z)).max() < 1e-8


def _tiny(seed=3):
    n_in, h, n_out, b = 5, 4, 3, 6
    shapes = mlp.sizes_of(n_in, h, n_out)
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(sum(int(np.prod(s)) for s in shapes)) * 0.7
    X = rng.standard_normal((b, n_in))
    T = rng.standard_normal((b, n_out))
    return p, shapes, X, T


def test_gradient_matches_central_differences():
    p, shapes, X, T = _tiny()
    loss, g = mlp.loss_grad(p, shapes, X, T, bf=False)
    fd = np.empty_like(p)
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd[i] = (mlp.loss_grad(p + e, shapes, X, T, bf=False)[0]
                 - mlp.loss_grad(p - e, shapes, X, T, bf=False)[0]) / 2e-6
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_loss_is_mean_squared_error_and_zero_at_the_target():
    p, shapes, X, _ = _tiny()
    for mode in (False, "weights"):
        Y, _ = mlp.forward(p, shapes, X, bf=mode)
        loss, g = mlp.loss_grad(p, shapes, X, Y, bf=mode)
        assert loss == 0.0 and np.abs(g).max() == 0.0
        loss2, _ = mlp.loss_grad(p, shapes, X, Y + 0.5, bf=mode)
        assert abs(loss2 - 0.25) < 1e-15


def test_weights_mode_is_fp64_on_bf16_weights():
    # the specification's reference: BF16 weights, everything else exact.  On weights that
    # already lie on the BF16 grid it is the FP64 network; biases are never rounded.
    p, shapes, X, T = _tiny()
    blocks = mlp.unpack(p, shapes)
    on_grid = mlp.pack([mlp.bf16(a) if i % 2 == 0 else a for i, a in enumerate(blocks)])
    Yw, _ = mlp.forward(p, shapes, X, bf="weights")
    Y0, _ = mlp.forward(on_grid, shapes, X, bf=False)
    assert np.array_equal(Yw, Y0)
    lw, gw = mlp.loss_grad(p, shapes, X, T, bf="weights")
    l0, g0 = mlp.loss_grad(on_grid, shapes, X, T, bf=False)
    assert lw == l0 and np.array_equal(gw, g0)
    # off the grid the weights move by at most 2^-8 relative, and so does a linear layer
    Yf, _ = mlp.forward(p, shapes, X, bf=False)
    assert 0.0 < np.abs(Yw - Yf).max() < 0.05 * np.abs(Yf).max()
    # the activation-rounding diagnostic differs from the reference
    Yb, _ = mlp.forward(p, shapes, X, bf=True)
    assert not np.array_equal(Yb, Yw)
    try:
        mlp.forward(p, shapes, X, bf="bogus")
    except ValueError:
        pass
    else:
        raise AssertionError("unknown mode accepted")


def test_bf16_mode_rounds_weights_and_layer_inputs():
    # with weights and inputs already on the BF16 grid and a linear-regime network the
    # two modes agree to the rounding of the hidden activations
    p, shapes, X, T = _tiny()
    Y, _ = mlp.forward(p, shapes, X, bf=False)
    Yb, _ = mlp.forward(p, shapes, X, bf=True)
    assert np.abs(Y - Yb).max() < 0.05 * np.abs(Y).max()
    pb, Xb = mlp.bf16(p), mlp.bf16(X)
    _, (A0, _, A1, _, A2) = mlp.forward(pb, shapes, Xb, bf=True)
    for A in (A0, A1, A2):
        assert np.array_equal(A, mlp.bf16(A))


def test_adam_first_step_is_a_signed_learning_rate_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -1e-3, 0.2])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    # second step with the same gradient: bias-corrected moments equal g and g^2 again
    p2, _, _ = mlp.adam_step(p1, g, m, v, 2, lr=0.01, eps=0.0)
    assert np.allclose(p2, p1 - 0.01 * np.sign(g), rtol=0, atol=1e-14)


def test_init_layout_and_scale():
    n_in, h, n_out = 7, 5, 3
    p = W.mlp_init(n_in, h, n_out, seed=1)
    shapes = mlp.sizes_of(n_in, h, n_out)
    assert p.dtype == np.float32 and len(p) == sum(int(np.prod(s)) for s in shapes)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, shapes)
    assert np.abs(W1).max() <= math.sqrt(6.0 / (n_in + h)) and not b1.any() and not b3.any()
    assert np.array_equal(p, W.mlp_init(n_in, h, n_out, seed=1))

"""Pins of the FP64 reference of the sidelobe network (CPU only)."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_exact_cases():
    one = 1.0
    cases = {one: one, one + 2 ** -8: one, one + 3 * 2 ** -9: one + 2 ** -7, one + 2 ** -7: one + 2 ** -7,
             one + 2 ** -8 + 2 ** -20: one + 2 ** -7, -2.5: -2.5, 0.0: 0.0}
    for x, want in cases.items():
        got = float(mlp.bf16_round(np.float32(x)))
        assert abs(got - want) <= 1e-7 * max(1.0, abs(want)), (x, got, want)
    # ties go to even mantissas: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7
    assert float(mlp.bf16_round(np.float32(1 + 3 * 2 ** -8))) == 1 + 2 ** -6


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    num = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(num - mlp.silu_grad(z)).max() < 1e-8


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    width, hidden, n = 16, 3, 9
    _, total = mlp.layout(width, hidden)
    p = rng.normal(0, 0.4, total)
    x = rng.normal(size=(n, 5))
    t = rng.normal(size=(n, 3))
    # straight-through rounding is the identity for the finite differences: check the exact network
    loss, g = mlp.loss_and_grad(p, x, t, width, hidden, round_weights=False)
    h = 1e-6
    idx = rng.choice(total, 60, replace=False)
    for i in idx:
        e = np.zeros(total)
        e[i] = h
        lp, _ = mlp.loss_and_grad(p + e, x, t, width, hidden, round_weights=False)
        lm, _ = mlp.loss_and_grad(p - e, x, t, width, hidden, round_weights=False)
        assert abs((lp - lm) / (2 * h) - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    z = np.zeros(50)
    new, m, v = mlp.adam_step(p, z, z, g, 1, 1e-3, 0.9, 0.999, 1e-12)
    assert np.abs((p - new) - 1e-3 * np.sign(g)).max() < 1e-12
    # second step with the same gradient keeps the signed step
    new2, _, _ = mlp.adam_step(new, m, v, g, 2, 1e-3, 0.9, 0.999, 1e-12)
    assert np.abs((new - new2) - 1e-3 * np.sign(g)).max() < 1e-12


def test_layout_counts():
    lay, total = mlp.layout(256, 4)
    assert total == 5 * 256 + 256 + 3 * (256 * 256 + 256) + 3 * 256 + 3
    assert lay[0][:3] == (0, 256, 5) and lay[-1][1:3] == (3, 256)

"""Pins of the fp64 reference of the branching network: central differences
(exact network, and the bf16 network at a point where its rounding is the
identity), bf16 rounding against its IEEE definition and torch's converter,
and the closed form of Adam's first step."""
import numpy as np
import torch

from oracle import mlp_ref as M


def test_exact_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    th = M.init_theta(1).astype(np.float64)
    X = rng.normal(0, 1, (80, M.F))
    # keep rows whose pre-activations stay clear of the ReLU kink, so that a
    # central difference of step h never crosses it
    _, pre, _ = M.forward(th, X, False)
    X = X[np.min(np.abs(pre), axis=1) > 0.01][:40]
    T = rng.normal(0, 1, X.shape[0])
    assert X.shape[0] >= 10
    g = M.grad(th, X, T, quantized=False)
    h = 1e-4
    num = np.zeros_like(g)
    for i in range(M.NP):
        e = np.zeros(M.NP)
        e[i] = h
        num[i] = (M.loss(th + e, X, T, False) - M.loss(th - e, X, T, False)) / (2 * h)
    err = np.abs(g - num) / np.maximum(1e-3, np.abs(num))
    assert err.max() < 1e-6


def test_bf16_rounding_definition():
    one = np.float32(1.0)
    ulp = 2.0 ** -7  # bf16 keeps 7 fraction bits
    cases = {
        1.0: 0x3F80,
        1.0 + ulp: 0x3F81,
        1.0 + ulp / 2: 0x3F80,            # tie -> even
        1.0 + 3 * ulp / 2: 0x3F82,        # tie -> even
        1.0 + ulp / 2 + 2 ** -20: 0x3F81,  # just above the tie
        -2.0: 0xC000,
        0.0: 0x0000,
    }
    for x, bits in cases.items():
        assert int(M.bf16_bits(np.float32(x))) == bits, x
    assert one == 1.0


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = (rng.normal(0, 10, 20000)).astype(np.float32)
    ours = M.bf16_value(M.bf16_bits(x))
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    th = rng.normal(0, 1, M.NP)
    g = rng.normal(0, 1, M.NP)
    new, m, v = M.adam_step(th, np.zeros(M.NP), np.zeros(M.NP), g, lr=0.01, step=1)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_quantized_forward_close_to_exact():
    rng = np.random.default_rng(3)
    th = M.init_theta(4)
    X = rng.uniform(0, 1, (100, M.F))
    yq, _, _ = M.forward(th, X, True)
    ye, _, _ = M.forward(th, X, False)
    assert np.max(np.abs(yq - ye)) < 0.05 * (1 + np.max(np.abs(ye)))


def test_quantized_gradient_at_bf16_exact_point():
    """grad(quantized=True) treats the bf16 rounding of weights, inputs and
    hidden activations as the identity.  At a point where every one of those
    values is already a bf16 number the rounding IS the identity, so there
    the straight-through gradient must equal the true derivative of the
    loss, measured by central differences of the exact network."""
    rng = np.random.default_rng(6)
    th = np.zeros(M.NP)
    # quarters, sixteenths and eighths: every weight, input and
    # pre-activation (|pre| <= 6.5, a multiple of 1/16) has at most 8
    # significant bits, so it is a bf16 number
    th[M.OFF_W1:M.OFF_B1] = rng.integers(-4, 5, M.H * M.F) / 4.0
    th[M.OFF_B1:M.OFF_W2] = rng.integers(-8, 9, M.H) / 16.0
    th[M.OFF_W2:M.OFF_B2] = rng.integers(-4, 5, M.H) / 8.0
    th[M.OFF_B2] = 0.125
    X = rng.integers(0, 5, (200, M.F)) / 4.0
    W1, b1, w2, _ = M.unpack(th)
    for a in (W1, b1, w2, X):
        assert np.array_equal(M.bf16_round(a), a)
    _, pre, Hact = M.forward(th, X, quantized=False)
    assert np.array_equal(M.bf16_round(Hact), Hact)
    # rows away from the ReLU kink (a step of 1e-4 never crosses it)
    X = X[np.min(np.abs(pre), axis=1) >= 1.0 / 16][:60]
    assert X.shape[0] >= 20
    T = rng.integers(-16, 17, X.shape[0]) / 8.0
    yq, _, _ = M.forward(th, X, quantized=True)
    ye, _, _ = M.forward(th, X, quantized=False)
    assert np.array_equal(yq, ye)
    g = M.grad(th, X, T, quantized=True)
    h = 1e-4
    num = np.zeros(M.NP)
    for i in range(M.NP):
        e = np.zeros(M.NP)
        e[i] = h
        num[i] = (M.loss(th + e, X, T, False) - M.loss(th - e, X, T, False)) / (2 * h)
    err = np.abs(g - num) / np.maximum(1e-3, np.abs(num))
    assert err.max() < 1e-6

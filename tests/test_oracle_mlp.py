"""Pins of the FP64 network reference (oracle/mlp.py) against things other than itself.

* a one-unit network evaluated by hand;
* the analytic gradient against central finite differences of the loss;
* BF16 rounding of hand-picked FP32 bit patterns (ties to even, carries into the exponent);
* the first Adam step, which moves every parameter by lr times the sign of its gradient;
* planted mistakes in a copy of the reference fail the finite-difference pin.
"""
import importlib.util
import os

import numpy as np
import pytest

from oracle import mlp as om


def test_one_unit_network_by_hand():
    # W1=2, b1=0.5, W2=3, b2=-1, W3=0.5, b3=0.25
    p = np.array([2.0, 0.5, 3.0, -1.0, 0.5, 0.25])
    x = np.array([[1.0], [-1.0]])
    y, _ = om.forward(p, x, (1, 1, 1))
    # x = 1: z1 = 2.5, z2 = 6.5, y = 3.25 + 0.25; x = -1: both ReLUs are off, y = b3
    assert y[:, 0].tolist() == [3.5, 0.25]
    t = np.array([[3.0], [0.0]])
    assert om.loss(p, x, t, None, (1, 1, 1)) == pytest.approx((0.5 ** 2 + 0.25 ** 2) / 2, abs=0)
    L, g = om.loss_and_grad(p, x, t, None, (1, 1, 1))
    # only the first row is active: dL/dy = 2 (0.5) / 2 = 0.5, dL/db3 adds 2 (0.25) / 2
    assert g[5] == pytest.approx(0.5 + 0.25)
    assert g[4] == pytest.approx(0.5 * 6.5)            # dL/dW3 = dy h2
    assert g[2] == pytest.approx(0.5 * 0.5 * 2.5)      # dL/dW2 = dy W3 h1
    assert g[0] == pytest.approx(0.5 * 0.5 * 3.0 * 1)  # dL/dW1 = dy W3 W2 x


def _fd_check(mod, dims=(3, 5, 2), n=7, seed=4):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.7, om.param_count(*dims))
    x = rng.normal(size=(n, dims[0]))
    t = rng.normal(size=(n, dims[2]))
    w = rng.uniform(0.5, 2.0, size=(n, dims[2]))
    _, g = mod.loss_and_grad(p, x, t, w, dims)
    fd = np.empty_like(p)
    h = 1e-6
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (om.loss(p + e, x, t, w, dims) - om.loss(p - e, x, t, w, dims)) / (2 * h)
    return np.max(np.abs(g - fd)) / np.max(np.abs(fd))


def test_gradient_matches_finite_differences():
    assert _fd_check(om) < 1e-7


@pytest.mark.parametrize("dims", [(8, 16, 6), (1, 4, 1)])
def test_gradient_matches_finite_differences_other_shapes(dims):
    assert _fd_check(om, dims=dims, n=11, seed=9) < 1e-7


def test_bf16_rounding_bit_patterns():
    f = np.float32
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20,
                     f(0.1), -2.0 ** -130, 2.0 - 2.0 ** -9, 65504.0], dtype=np.float64)
    want = [1.0,                 # exact
            1.0,                 # tie, even neighbour is 1
            1 + 2.0 ** -6,       # tie between 1+2^-7 (odd) and 1+2^-6 (even)
            1 + 2.0 ** -7,       # just above the tie
            0.10009765625,       # 0x3DCCCCCD -> 0x3DCD
            -2.0 ** -130,        # subnormal FP32 with a short significand stays exact
            2.0,                 # tie 2-2^-8 / 2: rounds up into the next binade (even)
            65536.0]             # 65504 = 1.999 * 2^15 rounds to 2^16
    assert om.bf16_round(vals).tolist() == want


def test_first_adam_step_moves_by_lr_sign():
    rng = np.random.default_rng(1)
    # |g| >= 1e-2, so eps / |g| <= 1e-6 keeps each step within 1e-8 of lr sign(g)
    g = rng.choice([-1.0, 1.0], 50) * 10.0 ** rng.uniform(-2, 3, 50)
    p = rng.normal(size=50)
    p1, m, v = om.adam_step(p, g, np.zeros(50), np.zeros(50), 1, 0.01)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1.1e-8)
    # a second step with the same gradient moves by the same amount again
    p2, _, _ = om.adam_step(p1, g, m, v, 2, 0.01)
    np.testing.assert_allclose(p2, p - 0.02 * np.sign(g), rtol=0, atol=2.2e-8)


MUTANTS = {
    "relu_mask_dropped_layer2": ("dz2 = (dy @ _q(W3, bf16).T) * (z2 > 0)",
                                 "dz2 = (dy @ _q(W3, bf16).T)"),
    "mask_from_wrong_layer": ("dz1 = (dz2 @ _q(W2, bf16).T) * (z1 > 0)",
                              "dz1 = (dz2 @ _q(W2, bf16).T) * (z2 > 0)"),
    "transposed_weight": ("dz1 = (dz2 @ _q(W2, bf16).T)", "dz1 = (dz2 @ _q(W2, bf16))"),
    "loss_scale": ("dy = 2.0 * w * e / y.size", "dy = w * e / y.size"),
    "weights_dropped": ("dy = 2.0 * w * e / y.size", "dy = 2.0 * e / y.size"),
    "bias_grad_wrong_axis": ("gb2, dz2 = dz2.sum(0), _q(dz2, bf16)",
                             "gb2, dz2 = dz2.mean(0), _q(dz2, bf16)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_finite_difference_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(om.__file__).read()
    assert src.count(old) == 1, name
    path = os.path.join(tmp_path, f"mlp_{name}.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"mlp_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    errs = [_fd_check(mod, dims=d, n=9, seed=3) for d in [(3, 5, 2), (4, 6, 3)]]
    assert max(errs) > 1e-3, name

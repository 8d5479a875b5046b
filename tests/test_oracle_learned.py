"""Pins for the oracle's parameter predictor, features and schedule driver.

The predictor stands in for the paper's regressor (Sec. VI); it maps five
instance features and the trade-off weight beta of Eq. 7 to (palette
fraction, list multiplier).  Pins: gradients
against central finite differences, the forward pass against the collapsed
affine map when every ReLU is active, Adam's first step in closed form,
feature values against direct counts and special cases.
"""
import math

import numpy as np
import pytest

from paper_2401_06713_amd import workloads as wl


def rand_params(orc, seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, orc.mlp_nparams())


def split(orc, p):
    H, I, O = orc.MLP_HIDDEN, orc.MLP_IN, orc.MLP_OUT
    sizes = [H * I, H, H * H, H, O * H, O]
    parts = np.split(p, np.cumsum(sizes)[:-1])
    return parts[0].reshape(H, I), parts[1], parts[2].reshape(H, H), parts[3], parts[4].reshape(O, H), parts[5]


def scaled(raw):
    return raw / np.array([16.0, 128.0, 128.0, 1.0, 16.0, 1.0])


def test_param_count(orc):
    assert orc.mlp_nparams() == 64 * 6 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def test_forward_zero_weights_gives_bias(orc):
    p = np.zeros(orc.mlp_nparams())
    p[-2:] = [0.7, -1.3]
    out = orc.mlp_forward(p, np.random.default_rng(0).random((5, 6)))
    assert np.allclose(out, [[0.7, -1.3]] * 5)


def test_forward_matches_affine_map_when_all_units_active(orc):
    rng = np.random.default_rng(1)
    p = np.abs(rng.normal(0, 0.2, orc.mlp_nparams()))  # positive weights, positive inputs: every ReLU passes
    raw = rng.random((7, 6)) * np.array([16, 128, 128, 1, 16, 1])
    W1, b1, W2, b2, W3, b3 = split(orc, p)
    expect = (W3 @ (W2 @ (W1 @ scaled(raw).T + b1[:, None]) + b2[:, None]) + b3[:, None]).T
    assert np.allclose(orc.mlp_forward(p, raw), expect, rtol=1e-12)


def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(2)
    p = rand_params(orc, 3)
    raw = rng.random((6, 6)) * np.array([16, 128, 60, 1, 8, 1])
    t = rng.normal(0, 1, (6, 2))
    _, g = orc.mlp_loss_grad(p, raw, t)
    idx = rng.choice(p.shape[0], 60, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (orc.mlp_loss_grad(pp, raw, t)[0] - orc.mlp_loss_grad(pm, raw, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd), abs(g[i])), (i, fd, g[i])


def test_loss_value(orc):
    p = np.zeros(orc.mlp_nparams())
    raw = np.ones((4, 6))
    t = np.array([[1.0, 2.0]] * 4)
    loss, _ = orc.mlp_loss_grad(p, raw, t)
    assert math.isclose(loss, 0.5 * (1 + 4))  # mean over rows of half squared error


def test_adam_first_step_closed_form(orc):
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    orc.adam_step(p, g, m, v, 1, lr=0.01)
    assert np.allclose(p, np.array([1.0, -2.0, 0.5]) - 0.01 * g / (np.abs(g) + 1e-8))


def test_squash_ranges(orc):
    assert np.allclose(orc.mlp_squash([0.0, 0.0]), (0.13, 2.5))
    f, a = orc.mlp_squash([-50.0, 50.0])
    assert math.isclose(f, 0.01, rel_tol=1e-9) and math.isclose(a, 4.0, rel_tol=1e-9)


def test_features_direct_counts(orc):
    x, z = wl.pauli_strings(3000, 40, (0.7, 0.1, 0.1, 0.1), seed=4)
    ids = np.sort(np.random.default_rng(0).choice(3000, 2000, replace=False)).astype(np.int32)
    f = orc.features(x, z, 40, ids, 9, 3, 0)
    assert math.isclose(f[0], math.log(2000))
    assert f[1] == 40 and f[4] == 3
    weight = np.bitwise_count(x[ids] | z[ids]).sum()
    assert math.isclose(f[2], weight / 2000)
    # iid strings: density near rho = (1 - (1 - 2p)^q) / 2, p = 6 * 0.01
    rho = (1 - (1 - 2 * 0.06) ** 40) / 2
    assert abs(f[3] - rho) < 5 * math.sqrt(rho * (1 - rho) / 4096)


def test_features_special_cases(orc):
    x, z = wl.majorana_strings(20)
    ids = np.arange(40, dtype=np.int32)
    assert orc.features(x, z, 20, ids, 1, 1, 0)[3] == 1.0  # every sampled pair anticommutes (pairs are distinct)
    x, z = wl.iz_strings(300, 12, seed=2)
    ids = np.arange(300, dtype=np.int32)
    assert orc.features(x, z, 12, ids, 1, 1, 0)[3] == 0.0
    assert orc.features(x, z, 12, ids, 1, 1, 1)[3] == 0.0
    assert orc.features(x, z, 12, ids[:1], 1, 1, 0)[3] == 0.0  # fewer than two vertices


@pytest.mark.parametrize("rel", [0, 1])
def test_constant_schedule_equals_fixed_parameters(orc, rel):
    x, z = wl.pauli_strings(700, 20, (0.6, 0.1, 0.2, 0.1), seed=5)
    a = orc.color(x, z, 20, 3, 0.1, 2.5, rel)
    b = orc.color_schedule(x, z, 20, 3, [0.1], [2.5], rel)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_schedule_uses_per_iteration_values(orc):
    x, z = wl.pauli_strings(800, 16, seed=6)
    nc, col, st = orc.color_schedule(x, z, 16, 1, [0.05, 0.2, 0.25], [3.0, 1.0, 2.0], 0)
    assert st[0]["P"] == math.ceil(0.05 * 800)
    assert st[1]["P"] == math.ceil(0.2 * st[1]["m"])
    for s in st[2:]:
        assert s["P"] == max(1, math.ceil(0.25 * s["m"]))

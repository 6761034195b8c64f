"""Pins of the oracle MLP (forward, hand-written backward, Adam, features)."""
import numpy as np

from oracle import mlp


def _data(seed, n=6):
    g = np.random.default_rng(seed)
    theta = mlp.init_params(g)
    P = mlp.unpack(theta)
    P["b1"][...] = g.uniform(-0.2, 0.2, 64)
    P["b2"][...] = g.uniform(-0.2, 0.2, 64)
    P["b3"][...] = g.uniform(-0.2, 0.2, 2)
    X = g.uniform(-2, 0, size=(n, 32))
    T = g.uniform(0, 1, size=(n, 2))
    return theta, X, T


def test_parameter_count():
    assert mlp.NPARAMS == 64 * 32 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 6402


def test_backward_matches_central_differences():
    """Every component of the hand-written gradient against a central finite
    difference (h = 1e-6); inputs are chosen so that no pre-activation lies
    within reach of the ReLU kink."""
    for seed in range(20):
        theta, X, T = _data(seed)
        _, c = mlp.forward(theta, X)
        if min(np.abs(c["z1"]).min(), np.abs(c["z2"]).min()) > 1e-3:
            break
    L, g = mlp.backward(theta, X, T)
    h = 1e-6
    fd = np.empty_like(g)
    for i in range(mlp.NPARAMS):
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd[i] = (mlp.loss(mlp.forward(tp, X)[0], T) - mlp.loss(mlp.forward(tm, X)[0], T)) / (2 * h)
    scale = np.abs(g).max()
    assert np.abs(fd - g).max() <= 1e-7 * scale
    assert L == mlp.loss(mlp.forward(theta, X)[0], T)


def test_forward_linear_special_case():
    """With W1 = [I; 0], W2 = I, zero biases and non-negative inputs the
    hidden layers pass x through, so y = W3[:, :32] x + b3."""
    theta = np.zeros(mlp.NPARAMS)
    P = mlp.unpack(theta)
    P["W1"][:32, :32] = np.eye(32)
    P["W2"][...] = np.eye(64)
    g = np.random.default_rng(3)
    P["W3"][...] = g.standard_normal((2, 64))
    P["b3"][...] = [0.5, -1.0]
    X = g.uniform(0, 1, size=(4, 32))
    y, _ = mlp.forward(theta, X)
    np.testing.assert_allclose(y, X @ P["W3"][:, :32].T + P["b3"], rtol=1e-14)


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected moments are g and g^2,
    so the update is -lr g / (|g| + eps)."""
    g = np.array([3.0, -2e-4, 0.0, 1e-9])
    theta, m, v = mlp.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    np.testing.assert_allclose(theta, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_features_of_a_geometric_profile():
    j = np.arange(1, 33)
    for rho in (1 / 16, 1 / 8, 1 / 2):
        f = mlp.features(10.0 ** (-rho * j))[0]
        np.testing.assert_allclose(f, -rho * (j - 1), atol=1e-12)
    assert np.all(mlp.features(np.zeros(32)) == 0.0)
    assert mlp.features(np.r_[1.0, np.zeros(31)])[0, 1] == -30.0


def test_predicted_widths_round_up():
    k, l = mlp.predict_widths(np.array([[10.2 / 32, 14.5 / 48], [1.0, 1.0], [0.0, 0.0]]))
    assert list(k) == [12, 32, 1]
    assert list(l) == [16, 40, 16]


def test_rank_label_closed_form_of_geometric_profiles():
    """Labels of the decaying-face workload (s_j = 10^(-rho j), j = 1..32)
    against the closed form of the geometric tail: the energy rule holds iff
    q^k <= tau^2 + (1 - tau^2) q^32 with q = 10^(-2 rho)."""
    tau = 1e-4
    seen = set()
    for rho in np.linspace(1 / 16, 1 / 2, 57):
        q = 10.0 ** (-2 * rho)
        x = np.log(tau ** 2 + (1 - tau ** 2) * q ** 32) / np.log(q)
        if min(x - np.floor(x), np.ceil(x) - x) < 1e-6:
            continue
        k = min(int(np.ceil(x)), 32)
        assert mlp.rank_label(10.0 ** (-rho * np.arange(1, 33)), tau) == k
        seen.add(k)
    assert len(seen) > 15

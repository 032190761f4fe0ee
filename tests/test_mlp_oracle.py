"""Pins of the FP64 cost-model MLP oracle (CPU): finite differences and closed forms."""
import numpy as np

from oracle import mlp


def _setup(seed=0, n=40, F=7, H=9):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(mlp.n_params(F, H)) * 0.5
    X = rng.standard_normal((n, F))
    t = rng.standard_normal(n)
    mean, std = rng.standard_normal(F), rng.uniform(0.5, 2.0, F)
    return theta, X, t, F, H, mean, std


def test_gradient_matches_finite_differences():
    theta, X, t, F, H, mean, std = _setup()
    g = mlp.gradient(theta, X, t, F, H, mean, std)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (mlp.loss(theta + e, X, t, F, H, mean, std) - mlp.loss(theta - e, X, t, F, H, mean, std)) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_forward_closed_form_linear_region():
    """With non-negative weights and inputs every ReLU is active: the net is affine."""
    F, H = 3, 4
    rng = np.random.default_rng(2)
    theta = np.abs(rng.standard_normal(mlp.n_params(F, H)))
    W1, b1, W2, b2, w3, b3 = mlp.unpack(theta, F, H)
    X = np.abs(rng.standard_normal((5, F)))
    y, _ = mlp.forward(theta, X, F, H)
    expect = ((X @ W1.T + b1) @ W2.T + b2) @ w3 + b3[0]
    np.testing.assert_allclose(y, expect, rtol=1e-13)


def test_adam_first_step_is_signed_lr():
    """From zero moments the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 2e-3, 0.0])
    th, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), step=1, lr=0.1)
    np.testing.assert_allclose(th, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_forward_hand_computed_with_clipped_units():
    """A 1-input, 2-unit network evaluated by hand, with ReLUs that clip and standardisation.

    W1 = [[1], [-1]], b1 = 0; W2 = [[1, 1], [-1, 0]], b2 = [0, 0.5]; w3 = [3, 5], b3 = -1;
    mean 1, std 2.
      x = 5:  x' = 2,  z1 = [2, -2] -> h1 = [2, 0],  z2 = [2, -1.5] -> h2 = [2, 0],  y = 5
      x = -5: x' = -3, z1 = [-3, 3] -> h1 = [0, 3],  z2 = [3, 0.5]  -> h2 = [3, 0.5], y = 10.5
    """
    theta = np.array([1.0, -1.0, 0.0, 0.0, 1.0, 1.0, -1.0, 0.0, 0.0, 0.5, 3.0, 5.0, -1.0])
    assert theta.size == mlp.n_params(1, 2)
    y, _ = mlp.forward(theta, np.array([[5.0], [-5.0]]), 1, 2, mean=[1.0], std=[2.0])
    np.testing.assert_allclose(y, [5.0, 10.5], rtol=0, atol=1e-15)
    # and the loss against targets [4, 10.5] is ((5-4)^2 + 0) / 2
    assert mlp.loss(theta, np.array([[5.0], [-5.0]]), [4.0, 10.5], 1, 2, [1.0], [2.0]) == 0.5


def test_adam_impulse_response_tells_beta1_from_beta2():
    """A gradient g at step 1 and 0 at step 2.  Solving the moment recursions by hand:
    m2 = b1 (1 - b1) g and v2 = b2 (1 - b2) g^2, so after bias correction
    m2 / (1 - b1^2) = b1 g / (1 + b1) and v2 / (1 - b2^2) = b2 g^2 / (1 + b2); the second
    step is lr * sign(g) * (b1 / (1 + b1)) / sqrt(b2 / (1 + b2)) (eps aside).  With
    b1 = 0.9, b2 = 0.999 that factor is 0.67006; with the two rates swapped it would be
    0.7261..., so the pin separates them (the first step, lr * sign(g), cannot)."""
    b1, b2, lr = 0.9, 0.999, 0.01
    g = np.array([2.5, -0.4])
    th, m, v = mlp.adam(np.zeros(2), g, np.zeros(2), np.zeros(2), step=1, lr=lr)
    th, m, v = mlp.adam(th, np.zeros(2), m, v, step=2, lr=lr)
    factor = (b1 / (1 + b1)) / np.sqrt(b2 / (1 + b2))
    assert abs(factor - 0.6700583) < 1e-6
    np.testing.assert_allclose(th, -lr * np.sign(g) * (1 + factor), rtol=1e-6)
    swapped = (b2 / (1 + b2)) / np.sqrt(b1 / (1 + b1))
    assert abs(swapped - factor) > 0.05


def test_splitmix64_published_outputs():
    """The first three outputs of SplitMix64 seeded with 0 (Steele, Lea, Flood 2014; the
    test vector quoted with the published generator): output k comes from state k * golden."""
    golden = 0x9E3779B97F4A7C15
    got = [mlp.splitmix64((k * golden) & ((1 << 64) - 1)) for k in range(3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_epoch_orders_are_permutations_and_change_per_epoch():
    orders = mlp.epoch_orders(50, 3, seed=42)
    assert len(orders) == 3
    for o in orders:
        assert sorted(o) == list(range(50))
    assert orders[0] != orders[1] != orders[2]
    assert mlp.epoch_orders(1, 2, seed=7) == [[0], [0]]
    assert mlp.epoch_orders(50, 1, seed=42)[0] == orders[0]
    # a different seed gives a different order
    assert mlp.epoch_orders(50, 1, seed=43)[0] != orders[0]


def test_epoch_orders_cover_every_permutation_of_three():
    """Fisher-Yates draws every permutation: over many seeds all 3! orders of 3 samples occur
    with roughly equal frequency (each 1/6)."""
    counts = {}
    for seed in range(3000):
        o = tuple(mlp.epoch_orders(3, 1, seed)[0])
        counts[o] = counts.get(o, 0) + 1
    assert len(counts) == 6
    assert all(abs(c / 3000 - 1 / 6) < 0.03 for c in counts.values()), counts


def test_train_with_one_full_batch_is_one_adam_step_on_all_samples():
    """With batch >= n and one epoch the shuffled order does not matter: the batch loss is the
    mean over all samples, so training is one Adam step with the full-data gradient."""
    theta, X, t, F, H, mean, std = _setup(seed=3, n=17)
    got = mlp.train(theta, X, t, F, H, mean, std, epochs=1, batch=64, lr=0.01, seed=9)
    g = mlp.gradient(theta, X, t, F, H, mean, std)
    want, _, _ = mlp.adam(theta, g, np.zeros_like(theta), np.zeros_like(theta), 1, 0.01)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


def test_train_batches_follow_the_epoch_order():
    """Two epochs of batches of 4 from 10 samples: 3 batches per epoch (4, 4, 2), six Adam steps,
    each on the samples the epoch's order puts in that batch."""
    theta, X, t, F, H, mean, std = _setup(seed=5, n=10)
    got = mlp.train(theta, X, t, F, H, mean, std, epochs=2, batch=4, lr=0.02, seed=11)
    th, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    step = 0
    for order in mlp.epoch_orders(10, 2, 11):
        for idx in (order[0:4], order[4:8], order[8:10]):
            step += 1
            th, m, v = mlp.adam(th, mlp.gradient(th, X[idx], t[idx], F, H, mean, std), m, v, step, 0.02)
    assert step == 6
    np.testing.assert_allclose(got, th, rtol=1e-12, atol=1e-15)

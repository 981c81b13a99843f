"""Pins of the float64 reference of the learned grouping (CPU only):
finite differences for its gradient, and for one-hot assignments the
expected F_D equals the oracle's occurrence F_D under the hard map."""
import numpy as np

import oracle
from oracle import learn_ref


def problem(seed, sigma=7, hidden=5, bits=4, n=40):
    rng = np.random.default_rng(seed)
    d_in = sigma + 3
    X = np.concatenate([np.eye(sigma), rng.random((sigma, 3))], axis=1)
    params = rng.normal(0, 0.7, learn_ref.n_params(d_in, hidden, bits))
    A = (rng.random((n, sigma)) < 0.4).astype(float)
    B = (rng.random((n, sigma)) < 0.4).astype(float)
    return X, params, hidden, bits, A, B


def test_gradient_matches_finite_differences():
    X, params, hidden, bits, A, B = problem(1)
    args = (hidden, bits, A, B, 1, 0.5, 2.0, 0.05)
    g = learn_ref.grads(X, params, *args)
    eps = 1e-6
    fd = np.zeros_like(params)
    for i in range(params.size):
        p1, p2 = params.copy(), params.copy()
        p1[i] += eps
        p2[i] -= eps
        fd[i] = (learn_ref.loss(X, p1, *args)[3] - learn_ref.loss(X, p2, *args)[3]) / (2 * eps)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_gradient_without_entropy_term_and_k2():
    X, params, hidden, bits, A, B = problem(2, sigma=9, hidden=6, bits=8, n=25)
    args = (hidden, bits, A, B, 2, 0.0, 3.0, 0.0)
    g = learn_ref.grads(X, params, *args)
    eps = 1e-6
    for i in np.random.default_rng(3).choice(params.size, 40, replace=False):
        p1, p2 = params.copy(), params.copy()
        p1[i] += eps
        p2[i] -= eps
        fd = (learn_ref.loss(X, p1, *args)[3] - learn_ref.loss(X, p2, *args)[3]) / (2 * eps)
        assert abs(g[i] - fd) <= 1e-5 * max(1.0, abs(fd))


def test_one_hot_expected_fd_is_occurrence_fd():
    """With one-hot P the model's expected distance is the popcount of the
    XOR of grouped occurrence fingerprints (Section 3.3) -- computed here by
    the oracle from the strings themselves."""
    rng = np.random.default_rng(4)
    letters = "etaoinshrdlu"
    sigma, bits = len(letters), 6
    field = rng.integers(0, bits + 1, size=sigma)  # bits = "no field"
    P = np.zeros((sigma, bits + 1))
    P[np.arange(sigma), field] = 1.0
    L = np.log(np.maximum(1.0 - P[:, :bits], learn_ref.CLAMP))
    words = ["".join(rng.choice(list(letters), size=int(rng.integers(1, 9)))) for _ in range(60)]
    M = np.array([[1.0 if c in w else 0.0 for c in letters] for w in words])
    mp = np.full(256, oracle.NONE, dtype=np.uint8)
    for i, c in enumerate(letters):
        if field[i] < bits:
            mp[ord(c)] = field[i]
    fps = oracle.fingerprints(words, oracle.OCC, 16, mp)
    ia, ib = rng.integers(0, 60, 200), rng.integers(0, 60, 200)
    E, _ = learn_ref.expected_fd(L, M[ia], M[ib])
    F = oracle.fd(fps[ia], fps[ib], oracle.OCC, 16)
    assert np.allclose(E, F, atol=1e-5)


def test_uniform_assignment_closed_form():
    """P uniform over B+1 outcomes: Z_S = (B/(B+1))^|S| per field."""
    sigma, bits = 5, 3
    P = np.full((sigma, bits + 1), 1.0 / (bits + 1))
    L = np.log(1.0 - P[:, :bits])
    A = np.array([[1, 1, 0, 0, 0.0]])
    B = np.array([[0, 1, 1, 1, 0.0]])
    q = bits / (bits + 1)
    expect = bits * (q ** 2 + q ** 3 - 2 * q ** 4)
    E, _ = learn_ref.expected_fd(L, A, B)
    assert np.isclose(E[0], expect)

"""Pins of the FP64 compression oracle (oracle/compression.py) against facts
that do not come from the oracle itself: the identity network, orthogonal
invariance of the full-spectrum kernel, rotation invariance of the
compressed features (equivariance of the per-l network with a norm gate),
finite differences of the training loss, and the closed-form PCA baseline."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synthetic
from oracle import compression as C


def small_coeffs(n_cells=2, seed_rot=None):
    b = synthetic.multi_species_cells().subset(list(range(n_cells)))
    h = b.hypers
    _, c, p = oracle.features(b)
    K, L2 = h["n_species"] * h["nmax"], (h["lmax"] + 1) ** 2
    return b, c.reshape(-1, K, L2), p.reshape(c.shape[0], h["lmax"] + 1, -1)


@pytest.fixture(scope="module")
def coeffs():
    return small_coeffs()


def random_weights(rng, K, Q, H, lmax, scale=0.3):
    parts = []
    for _ in range(lmax + 1):
        parts.append((rng.normal(size=(H, K)) * scale / np.sqrt(K), rng.normal(size=(Q, H)) * scale / np.sqrt(H),
                      rng.normal(size=H) * 0.5, rng.normal(size=H) * 0.5))
    return C.pack(parts)


def test_power_spectrum_matches_c_oracle(coeffs):
    _, c, p = coeffs
    assert np.abs(C.power_spectrum(c) - p).max() <= 1e-13 * np.abs(p).max()


def test_identity_network_reproduces_plain_spectrum(coeffs):
    """W1 = W2 = I, alpha = beta = 0: the gate 2 sigmoid(0) = 1, so c~ = c."""
    _, c, p = coeffs
    K, lmax = c.shape[1], int(np.sqrt(c.shape[2])) - 1
    w = C.pack([(np.eye(K), np.eye(K), np.zeros(K), np.zeros(K)) for _ in range(lmax + 1)])
    ct = C.compress(c, w, K, K)
    assert np.array_equal(ct, c)
    assert C.kernel_error(p, C.power_spectrum(ct)) <= 1e-14


def test_full_kernel_is_invariant_under_orthogonal_channel_maps(coeffs):
    """The linear kernel of the full symmetric spectrum depends on the
    channel space only through inner products, so any orthogonal W1 with
    W2 = I (gate off) leaves it unchanged -- the packed kernel would not."""
    _, c, p = coeffs
    K, lmax = c.shape[1], int(np.sqrt(c.shape[2])) - 1
    rng = np.random.default_rng(7)
    parts = []
    for _ in range(lmax + 1):
        U, _ = np.linalg.qr(rng.normal(size=(K, K)))
        parts.append((U, np.eye(K), np.zeros(K), np.zeros(K)))
    pt = C.power_spectrum(C.compress(c, C.pack(parts), K, K))
    assert C.kernel_error(p, pt) <= 1e-12


def test_compressed_features_are_rotation_invariant():
    """Rotating every position (and cell) leaves p~ unchanged for any
    weights: each layer acts on channels only and the gate sees |h| over m."""
    b = synthetic.multi_species_cells().subset([0])
    h = b.hypers
    K, L2 = h["n_species"] * h["nmax"], (h["lmax"] + 1) ** 2
    q, _ = np.linalg.qr(np.random.default_rng(11).normal(size=(3, 3)))
    b2 = synthetic.Batch(b.positions @ q.T, b.species, b.atom_offsets, b.cells @ q.T, b.pbc, b.hypers)
    _, c1, _ = oracle.features(b)
    _, c2, _ = oracle.features(b2)
    w = random_weights(np.random.default_rng(3), K, 16, 32, h["lmax"])
    p1 = C.power_spectrum(C.compress(c1.reshape(-1, K, L2), w, 16, 32))
    p2 = C.power_spectrum(C.compress(c2.reshape(-1, K, L2), w, 16, 32))
    assert np.abs(p1 - p2).max() <= 1e-10 * np.abs(p1).max()


def test_loss_gradient_matches_finite_differences(coeffs):
    _, c, p = coeffs
    c = c[:12]
    K, lmax = c.shape[1], int(np.sqrt(c.shape[2])) - 1
    Q, H = 4, 6
    rng = np.random.default_rng(5)
    w = random_weights(rng, K, Q, H, lmax, scale=1.0)
    Kref = C.linear_kernel(C.power_spectrum(c))
    L, g = C.loss_and_grad(c, Kref, w, Q, H)
    idx = rng.choice(w.size, 40, replace=False)
    for k in idx:
        e = 1e-6 * max(1.0, abs(w[k]))
        wp, wm = w.copy(), w.copy()
        wp[k] += e
        wm[k] -= e
        fd = (C.loss_and_grad(c, Kref, wp, Q, H)[0] - C.loss_and_grad(c, Kref, wm, Q, H)[0]) / (2 * e)
        assert abs(fd - g[k]) <= 1e-5 * abs(fd) + 1e-7 * np.abs(g).max(), (k, fd, g[k])


def test_pca_baseline_is_exact_at_full_rank_and_monotone(coeffs):
    _, c, p = coeffs
    K = c.shape[1]
    errs = []
    for Q in (4, 8, 16, 32, K):
        w = C.pca_weights(c, Q, max(Q, 16))
        errs.append(C.kernel_error(p, C.power_spectrum(C.compress(c, w, Q, max(Q, 16)))))
    assert errs[-1] <= 1e-12
    assert all(a >= b - 1e-12 for a, b in zip(errs, errs[1:])), errs


def test_adam_first_step_moves_by_lr_times_sign():
    """After bias correction the first Adam step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p, g = rng.normal(size=50), rng.normal(size=50)
    p1, m, v = C.adam_step(p, g, np.zeros(50), np.zeros(50), 1e-2, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(p - p1, 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)

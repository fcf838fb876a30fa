"""FP64 oracle of the learned channel compression -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  Plain numpy, double precision, written from the
definitions; it shares no code with the GPU library.

The compression maps the K = S * nmax (species, n) channels of the expansion
coefficients to Q contracted channels before the power spectrum: a learned
counterpart of the data-driven reduction of the feature space (Sec. 4.H;
the lossy strategy of Sec. 7) that keeps the symmetry of the features (the
abstract asks that reductions leave the symmetry properties intact).  For
every degree l the same two-layer network acts on the channel index of each
m-column of c, so a rotation (which mixes the m of one l) commutes with it:

    h_{l}   = W1_l c_{l}                      ([H x K] [K x (2l+1)])
    g_{l,q} = h_{l,q} * 2 sigmoid(alpha_{l,q} |h_{l,q}| + beta_{l,q})
                                              (|.| over m: a norm gate)
    c~_{l}  = W2_l g_{l}                      ([Q x H] [H x (2l+1)])
    p~_{l,q1<=q2} = sum_m c~_{q1,lm} c~_{q2,lm}

With alpha = beta = 0 the gate is the identity, so W1 = W2 = identity and
Q = H = K reproduce the plain power spectrum exactly.

Score (reading of the compressed-kernel error): the linear kernel of the
full symmetric power spectrum, K_ij = sum_{l,k1,k2} p_{lk1k2}(i) p_{lk1k2}(j)
(off-diagonal packed entries weighted 2), which does not depend on the
orthonormal basis of the channel space; K~_ij the same over p~;
eps_K = |K~ - K|_F / |K|_F on held-out centres.  Training minimises
L = |K~ - K|_F^2 / |K|_F^2 over batches.

Weights are one flat array, per l in order: W1_l [H][K], W2_l [Q][H],
alpha_l [H], beta_l [H].
"""
from __future__ import annotations

import numpy as np


def l_slices(lmax):
    return [slice(l * l, (l + 1) * (l + 1)) for l in range(lmax + 1)]


def n_params(K, Q, H, lmax):
    return (lmax + 1) * (H * K + Q * H + 2 * H)


def unpack(w, K, Q, H, lmax):
    """Per-l views (W1, W2, alpha, beta) of the flat weight array."""
    out, o = [], 0
    for _ in range(lmax + 1):
        W1 = w[o:o + H * K].reshape(H, K); o += H * K
        W2 = w[o:o + Q * H].reshape(Q, H); o += Q * H
        al = w[o:o + H]; o += H
        be = w[o:o + H]; o += H
        out.append((W1, W2, al, be))
    return out


def pack(parts):
    return np.concatenate([np.concatenate([W1.ravel(), W2.ravel(), al, be]) for W1, W2, al, be in parts])


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def power_spectrum(c):
    """p_{l,k1<=k2} = sum_m c_{k1,lm} c_{k2,lm}; c [N, K, L2] -> [N, lmax+1, K(K+1)/2]."""
    N, K, L2 = c.shape
    lmax = int(round(np.sqrt(L2))) - 1
    iu = np.triu_indices(K)
    out = np.empty((N, lmax + 1, len(iu[0])))
    for l, sl in enumerate(l_slices(lmax)):
        P = np.einsum("ikm,ijm->ikj", c[:, :, sl], c[:, :, sl])
        out[:, l, :] = P[:, iu[0], iu[1]]
    return out


def compress(c, w, Q, H):
    """c [N, K, L2] -> c~ [N, Q, L2] through the per-l network."""
    N, K, L2 = c.shape
    lmax = int(round(np.sqrt(L2))) - 1
    out = np.empty((N, Q, L2))
    for (W1, W2, al, be), sl in zip(unpack(w, K, Q, H, lmax), l_slices(lmax)):
        h = np.einsum("qk,ikm->iqm", W1, c[:, :, sl])
        nrm = np.sqrt(np.sum(h * h, axis=2))
        g = h * (2.0 * sigmoid(al[None, :] * nrm + be[None, :]))[:, :, None]
        out[:, :, sl] = np.einsum("pq,iqm->ipm", W2, g)
    return out


def full_weights(Q, lmax):
    """Weight of each packed feature in the linear kernel of the full
    (symmetric) power spectrum: 1 on k1 = k2, 2 on k1 < k2."""
    iu = np.triu_indices(Q)
    w = np.where(iu[0] == iu[1], 1.0, 2.0)
    return np.tile(w, lmax + 1)


def linear_kernel(p):
    """K_ij = sum_{l,k1,k2} p_{l k1 k2}(i) p_{l k1 k2}(j) over the full
    symmetric power spectrum (from the packed p [N, lmax+1, Q(Q+1)/2])."""
    N, lm1, F = p.shape
    Q = int(round((np.sqrt(8 * F + 1) - 1) / 2))
    P = p.reshape(N, -1)
    return (P * full_weights(Q, lm1 - 1)[None, :]) @ P.T


def kernel_error(p_full, p_comp):
    K, Kt = linear_kernel(p_full), linear_kernel(p_comp)
    return float(np.linalg.norm(Kt - K) / np.linalg.norm(K))


def loss_and_grad(c, Kref, w, Q, H):
    """L = |K~ - Kref|_F^2 / |Kref|_F^2 for the batch c and dL/dw, by the
    chain rule written out step by step (forward values kept)."""
    N, K, L2 = c.shape
    lmax = int(round(np.sqrt(L2))) - 1
    parts = unpack(w, K, Q, H, lmax)
    iu = np.triu_indices(Q)
    cache, pt = [], np.empty((N, lmax + 1, len(iu[0])))
    for l, ((W1, W2, al, be), sl) in enumerate(zip(parts, l_slices(lmax))):
        x = c[:, :, sl]
        h = np.einsum("qk,ikm->iqm", W1, x)
        nrm = np.sqrt(np.sum(h * h, axis=2))
        s = sigmoid(al[None, :] * nrm + be[None, :])
        g = h * (2.0 * s)[:, :, None]
        ct = np.einsum("pq,iqm->ipm", W2, g)
        P = np.einsum("ipm,iqm->ipq", ct, ct)
        pt[:, l, :] = P[:, iu[0], iu[1]]
        cache.append((x, h, nrm, s, g, ct))
    Pt = pt.reshape(N, -1)
    fw = full_weights(Q, lmax)[None, :]
    Kt = (Pt * fw) @ Pt.T
    norm2 = np.sum(Kref * Kref)
    D = Kt - Kref
    L = float(np.sum(D * D) / norm2)
    dKt = 2.0 * D / norm2
    dPt = ((dKt + dKt.T) @ Pt) * fw
    dpt = dPt.reshape(pt.shape)
    grads = []
    for l, ((W1, W2, al, be), (x, h, nrm, s, g, ct)) in enumerate(zip(parts, cache)):
        # p~_{q1 q2} = sum_m ct_{q1 m} ct_{q2 m} on q1 <= q2
        Gp = np.zeros((N, Q, Q))
        Gp[:, iu[0], iu[1]] = dpt[:, l, :]
        dct = np.einsum("ipq,iqm->ipm", Gp + np.transpose(Gp, (0, 2, 1)), ct)
        dW2 = np.einsum("ipm,iqm->pq", dct, g)
        dg = np.einsum("pq,ipm->iqm", W2, dct)
        # g = 2 s h, s = sigmoid(al |h| + be)
        ds = 2.0 * np.sum(dg * h, axis=2)
        dz = ds * s * (1.0 - s)
        dal = np.sum(dz * nrm, axis=0)
        dbe = np.sum(dz, axis=0)
        dnrm = dz * al[None, :]
        with np.errstate(invalid="ignore", divide="ignore"):
            dh_n = np.where(nrm[:, :, None] > 0, h / nrm[:, :, None], 0.0) * dnrm[:, :, None]
        dh = dg * (2.0 * s)[:, :, None] + dh_n
        dW1 = np.einsum("iqm,ikm->qk", dh, x)
        grads.append((dW1, dW2, dal, dbe))
    return L, pack(grads)


def pca_weights(c, Q, H):
    """Closed-form baseline: per l, project the channels on the top-Q
    eigenvectors of sum_{i,m} c_{:,lm} c_{:,lm}^T (W1 = [U^T; 0], W2 = [I 0],
    gate off)."""
    N, K, L2 = c.shape
    lmax = int(round(np.sqrt(L2))) - 1
    parts = []
    for sl in l_slices(lmax):
        x = c[:, :, sl]
        C = np.einsum("ikm,ijm->kj", x, x)
        ev, U = np.linalg.eigh(C)
        U = U[:, ::-1][:, :Q]
        W1 = np.zeros((H, K)); W1[:Q, :] = U.T
        W2 = np.zeros((Q, H)); W2[:, :Q] = np.eye(Q)
        parts.append((W1, W2, np.zeros(H), np.zeros(H)))
    return pack(parts)


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    """Adam (Kingma & Ba 2015, Algorithm 1) with bias correction; returns
    (p, m, v) after one step (step counts from 1)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

"""Packed MLP weight layout helpers shared by the learned-far-field GPU tests:
random weights in the library's packed layout (W1 [Kp x H] with rows >= K
unused, b1 [H], W2 [H x H], b2 [H], W3 [H x 16] with columns >= 3 unused,
b3 [16]) and their unpacking into the oracle's dict of FP64 matrices."""
import math

import numpy as np


def oracle_weights(w_packed, K, H):
    Kp = (K + 31) // 32 * 32
    o = 0
    W1 = w_packed[o:o + Kp * H].reshape(Kp, H)[:K]; o += Kp * H
    b1 = w_packed[o:o + H]; o += H
    W2 = w_packed[o:o + H * H].reshape(H, H); o += H * H
    b2 = w_packed[o:o + H]; o += H
    W3 = w_packed[o:o + H * 16].reshape(H, 16)[:, :3]; o += H * 16
    b3 = w_packed[o:o + 16][:3]
    return {k: np.asarray(v, np.float64) for k, v in
            dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3).items()}


def random_packed(nW, K, H, seed):
    rng = np.random.default_rng(seed)
    w = np.zeros(nW, np.float32)
    Kp = (K + 31) // 32 * 32
    o = 0
    w[o:o + Kp * H].reshape(Kp, H)[:K] = rng.standard_normal((K, H)) / math.sqrt(K); o += Kp * H
    w[o:o + H] = rng.standard_normal(H) * 0.1; o += H
    w[o:o + H * H] = rng.standard_normal(H * H) / math.sqrt(H); o += H * H
    w[o:o + H] = rng.standard_normal(H) * 0.1; o += H
    w[o:o + H * 16].reshape(H, 16)[:, :3] = rng.standard_normal((H, 3)) / math.sqrt(H); o += H * 16
    w[o:o + 3] = rng.standard_normal(3) * 0.1
    return w

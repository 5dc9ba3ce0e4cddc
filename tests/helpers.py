"""Shared test helpers: random canonical multi-word inputs and host/device moves."""
from fractions import Fraction

import numpy as np

from oracle.exact import canon


def rand_words(g, K, n, spread=3):
    """Random canonical K-word numbers: greedy rounding of random rationals
    carrying a few words more than K, exponents in [-spread, spread]."""
    out = np.zeros((K, n))
    for i in range(n):
        e = int(g.integers(-spread, spread + 1))
        q = Fraction(0)
        for w in range(K + 2):
            q += Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * w + e)
        out[:, i] = canon(q, K)
    return out


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()

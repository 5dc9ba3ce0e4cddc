"""The oracle's OpenMP loops change nothing but speed.

The LU updates, the U12 substitution, the split update and the matrix
product share out independent columns, the residual independent rows; each
entry still receives its operations in the order the serial definition
states (Kouya 2021, Sec. 2: LU with partial pivoting; Listing 1: residual).
So one thread and many threads must agree bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import synth


@pytest.fixture
def many_threads():
    default = O.set_threads(0)
    yield max(default, 4)
    O.set_threads(default)


def _both(fn, nthreads):
    O.set_threads(1)
    a = fn()
    O.set_threads(nthreads)
    b = fn()
    return a, b


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_lu_and_solve_independent_of_threads(K, many_threads):
    n = 150
    A, b, _ = synth.problem("randsvd", n, config=1, instance=K, cond=1e12)
    S = O.stage(K, A)
    (LU1, p1, i1), (LU2, p2, i2) = _both(lambda: O.getrf(K, S), many_threads)
    np.testing.assert_array_equal(LU1, LU2)
    np.testing.assert_array_equal(p1, p2)
    assert i1 == i2
    (Z1, Z2) = _both(lambda: O.getrs(K, LU1, p1, O.round_words(K, b)), many_threads)
    np.testing.assert_array_equal(Z1, Z2)


@pytest.mark.parametrize("K,s", [(2, 5), (3, 7)])
def test_split_lu_independent_of_threads(K, s, many_threads):
    n = 200
    A, _, _ = synth.problem("randsvd", n, config=1, instance=10 + K, cond=1e10)
    S = O.stage(K, A)
    (LU1, p1, _), (LU2, p2, _) = _both(lambda: O.getrf_ozaki(K, S, s), many_threads)
    np.testing.assert_array_equal(LU1, LU2)
    np.testing.assert_array_equal(p1, p2)


def test_residual_gemm_refine_independent_of_threads(many_threads):
    n = 120
    A, b, _ = synth.problem("uniform", n, config=0, instance=3)
    g = np.random.default_rng(5)
    x = np.zeros((4, n))
    x[0] = 1 + g.uniform(-1e-20, 1e-20, n)
    x[1] = g.uniform(-1e-40, 1e-40, n)
    r1, r2 = _both(lambda: O.residual(A, x, b), many_threads)
    np.testing.assert_array_equal(r1, r2)
    Am, Bm, Cm = (g.uniform(-1, 1, (3, 90, 70)), g.uniform(-1, 1, (3, 50, 90)), g.uniform(-1, 1, (3, 50, 70)))
    c1, c2 = _both(lambda: O.gemm(3, Am, Bm, Cm), many_threads)
    np.testing.assert_array_equal(c1, c2)
    f1, f2 = _both(lambda: O.refine(A, b, 2, ozaki=5), many_threads)
    np.testing.assert_array_equal(f1["x"], f2["x"])
    assert (f1["iters"], f1["status"]) == (f2["iters"], f2["status"])

"""GPU parity of the learned precision choice's kernels against the oracle:
the 24 features (bnc_features) of systems of order 1..256, and the MLP's
forward pass, gradient and Adam step (bnc_mlp_*) against the float64
oracle; the loss falls step by step on a fixed batch."""
import sys

import numpy as np
import pytest

import oracle.selector as OS
import synth
from helpers import dev, host

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_12550_amd as P
    return P


def systems():
    out = []
    sizes = [1, 2, 7, 33, 64, 100, 129, 200, 256, 257, 300, 512]
    for i, n in enumerate(sizes):
        kind = "uniform" if i % 2 else "randsvd"
        Ap, b, _ = synth.problem(kind, n, config=4, instance=i, cond=[1e2, 1e9, 1e15, 1e25][i % 4])
        out.append((Ap, b))
    # quad-double-word entries: the features read the leading words
    for i, n in enumerate((90, 280)):
        Ap, b, _ = synth.problem("randsvd_words", n, config=4, instance=40 + i, cond=1e40)
        out.append((Ap, b))
    g = np.random.default_rng(8)
    Z = g.uniform(-1, 1, (40, 40))
    Z[:, 7] = 0.0                                    # exactly singular
    D = np.diag(g.uniform(0.5, 2.0, 30))             # diagonal
    M = g.uniform(-1, 1, (50, 50))                   # symmetric
    for A in (Z, D, M + M.T):
        Ap = synth.planes(A)
        b, _ = synth.rhs_ones(Ap)
        out.append((Ap, b))
    return out


@pytest.mark.parametrize("slots", [0, 3])
def test_features_match_oracle(P, slots):
    sy = systems()
    ref = np.array([OS.features(Ap, b) for Ap, b in sy])
    say("features slots", slots, "systems", len(sy))
    F = host(P.features([dev(Ap) for Ap, _ in sy], [dev(b) for _, b in sy], slots=slots))
    assert F.shape == (len(sy), 24)
    r32 = ref.astype(np.float32)
    for k in (7, 16, 22):                            # counts and decisions: exact
        np.testing.assert_array_equal(F[:, k], r32[:, k], err_msg=f"feature {k}")
    np.testing.assert_allclose(F, r32, rtol=2e-6, atol=2e-5)


def test_mlp_forward_grad_adam_match_oracle(P):
    import torch
    g = np.random.default_rng(21)
    B = 257
    params = g.normal(0, 0.3, OS.NPARAM)
    X = g.normal(0, 3, (B, 24))
    norm = np.concatenate([g.normal(0, 1, 24), 1.0 / (1.0 + g.random(24))])
    cls = g.integers(0, 4, B)
    tgt = g.normal(2.0, 1.0, B)
    say("mlp parity")
    net = P.MLP(torch.tensor(params, dtype=torch.float32, device="cuda"),
                torch.tensor(norm, dtype=torch.float32, device="cuda"))
    p32 = params.astype(np.float32).astype(np.float64)
    n32 = norm.astype(np.float32).astype(np.float64)
    X32 = X.astype(np.float32).astype(np.float64)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    out = host(net.forward(Xt))
    ref_out = OS.forward(p32, X32, n32)[3]
    np.testing.assert_allclose(out, ref_out, rtol=1e-4, atol=1e-4 * np.abs(ref_out).max())
    loss = host(net.grad(Xt, torch.tensor(cls, device="cuda"), torch.tensor(tgt, device="cuda")))[0]
    ref_loss, ref_g = OS.loss_and_grad(p32, X32, n32, cls, tgt.astype(np.float32).astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    G = host(net.grads).astype(np.float64)
    assert np.linalg.norm(G - ref_g) <= 1e-3 * np.linalg.norm(ref_g)
    assert np.abs(G - ref_g).max() <= 1e-3 * np.abs(ref_g).max()
    net.adam(lr=1e-2)
    ref_p, _, _ = OS.adam(p32, G, np.zeros_like(G), np.zeros_like(G), 1, lr=1e-2)
    np.testing.assert_allclose(host(net.params), ref_p, rtol=1e-5, atol=1e-6)


def test_loss_decreases_on_a_fixed_batch(P):
    import torch
    g = np.random.default_rng(22)
    B = 512
    X = torch.tensor(g.normal(0, 1, (B, 24)), dtype=torch.float32, device="cuda")
    cls = torch.tensor(g.integers(0, 4, B), device="cuda")
    tgt = torch.tensor(g.normal(2.0, 0.5, B), dtype=torch.float32, device="cuda")
    norm = torch.tensor(np.concatenate([np.zeros(24), np.ones(24)]), dtype=torch.float32, device="cuda")
    net = P.MLP(torch.tensor(g.normal(0, 0.2, OS.NPARAM), dtype=torch.float32, device="cuda"), norm)
    say("mlp descent")
    losses = []
    for _ in range(25):
        losses.append(float(host(net.grad(X, cls, tgt))[0]))
        net.adam(lr=3e-3)
    assert all(b < a for a, b in zip(losses, losses[1:])), losses

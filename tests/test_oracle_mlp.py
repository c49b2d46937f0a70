"""Pins of the surrogate-network oracle: finite differences, closed forms, hand-built nets."""
import numpy as np
import pytest

from oracle import mlp as om


def _rand_params(rng, h1=8, h2=8, nk=5):
    return {"W1": rng.normal(size=(h1, 4)), "b1": rng.normal(size=h1) * 0.1,
            "W2": rng.normal(size=(h2, h1)) / np.sqrt(h1), "b2": rng.normal(size=h2) * 0.1,
            "w3": rng.normal(size=h2), "b3": np.array(0.3), "emb": rng.uniform(0, 1, nk)}


def _batch(rng, B=7, nk=5):
    return (rng.integers(0, nk, B), np.rint(2.0 ** rng.uniform(8, 26, B)).astype(np.int64),
            2 ** rng.integers(0, 11, B), rng.integers(1, 65, B), rng.normal(size=B))


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    p = _rand_params(rng)
    kid, N, bx, by, t = _batch(rng)
    _, g = om.loss_and_grads(p, kid, N, bx, by, t)
    h = 1e-6
    for name in om.PARAM_NAMES:
        flat = np.asarray(p[name], np.float64).reshape(-1)
        for i in range(flat.size):
            q = {k: np.array(v, np.float64, copy=True) for k, v in p.items()}
            qf = q[name].reshape(-1)
            qf[i] = flat[i] + h
            lp, _ = om.loss_and_grads(q, kid, N, bx, by, t)
            qf[i] = flat[i] - h
            lm, _ = om.loss_and_grads(q, kid, N, bx, by, t)
            fd = (lp - lm) / (2 * h)
            an = np.asarray(g[name]).reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, an)


def test_embedding_gradient_accumulates_per_kernel():
    """Samples of one kernel add up in its embedding's gradient; unused kernels get zero."""
    rng = np.random.default_rng(1)
    p = _rand_params(rng, nk=6)
    kid = np.array([2, 2, 4, 2])
    N, bx, by, t = np.array([1 << 10, 1 << 12, 1 << 14, 1 << 16]), np.array([1, 2, 4, 8]), \
        np.array([64, 32, 16, 8]), np.array([0.1, -0.2, 0.3, 0.0])
    _, g = om.loss_and_grads(p, kid, N, bx, by, t)
    assert g["emb"][0] == 0 and g["emb"][1] == 0 and g["emb"][3] == 0 and g["emb"][5] == 0
    parts = [om.loss_and_grads(p, kid[i:i + 1], N[i:i + 1], bx[i:i + 1], by[i:i + 1], t[i:i + 1])[1]["emb"]
             for i in range(4)]
    # the batch loss is the mean of the per-sample losses
    assert np.allclose(g["emb"], sum(parts) / 4.0, rtol=1e-12, atol=1e-15)


def test_hand_built_network_forward():
    """W1 picks the features, W2 = identity, w3 sums: y = relu-sum of the features."""
    p = {"W1": np.eye(4), "b1": np.zeros(4), "W2": np.eye(4), "b2": np.zeros(4),
         "w3": np.ones(4), "b3": np.array(0.5), "emb": np.array([0.25, -3.0])}
    y, _ = om.forward(p, np.array([0, 1]), np.array([1 << 13, 1 << 26]), np.array([1 << 5, 1]),
                      np.array([1 << 10, 1 << 2]))
    # sample 0: 13/26 + 5/10 + 10/10 + 0.25 + 0.5; sample 1: 1 + 0 + 0.2 + relu(-3) + 0.5
    assert np.allclose(y, [0.5 + 0.5 + 1.0 + 0.25 + 0.5, 1.0 + 0.0 + 0.2 + 0.0 + 0.5], rtol=0, atol=1e-15)


def test_adam_first_step_is_signed_learning_rate():
    """From zero moments, bias correction gives m_hat = g, v_hat = g^2: the step is
    -lr g / (|g| + eps), i.e. -lr sign(g) up to eps."""
    rng = np.random.default_rng(2)
    p = _rand_params(rng)
    g = {k: rng.normal(size=np.shape(v)) for k, v in p.items()}
    p2, m2, v2 = om.adam_step(p, g, om.zeros_like(p), om.zeros_like(p), 1, lr=1e-3)
    for k in om.PARAM_NAMES:
        d = np.asarray(p2[k]) - np.asarray(p[k])
        assert np.allclose(d, -1e-3 * np.asarray(g[k]) / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=1e-18)
        assert np.allclose(m2[k], 0.1 * np.asarray(g[k]))
        assert np.allclose(v2[k], 0.001 * np.asarray(g[k]) ** 2)


def test_adam_constant_gradient_moments():
    """With a constant gradient g the bias-corrected moments stay exactly g and g^2."""
    p = {k: np.zeros(3) for k in om.PARAM_NAMES}
    g = {k: np.array([0.5, -2.0, 1e-3]) for k in om.PARAM_NAMES}
    m, v = om.zeros_like(p), om.zeros_like(p)
    for s in range(1, 6):
        p, m, v = om.adam_step(p, g, m, v, s, lr=0.01)
    expect = -5 * 0.01 * g["W1"] / (np.abs(g["W1"]) + 1e-8)
    for k in om.PARAM_NAMES:
        assert np.allclose(p[k], expect, rtol=1e-9)


@pytest.mark.parametrize("seed", [3, 4])
def test_training_reduces_loss_on_a_learnable_target(seed):
    """Plain gradient steps on a target the network can represent lower the loss."""
    rng = np.random.default_rng(seed)
    p = _rand_params(rng, h1=16, h2=16)
    kid, N, bx, by, _ = _batch(rng, B=64)
    t = np.log2(N) / 26.0 - np.log2(bx) / 10.0
    l0, _ = om.loss_and_grads(p, kid, N, bx, by, t)
    m, v = om.zeros_like(p), om.zeros_like(p)
    for s in range(1, 201):
        _, g = om.loss_and_grads(p, kid, N, bx, by, t)
        p, m, v = om.adam_step(p, g, m, v, s, lr=1e-2)
    l1, _ = om.loss_and_grads(p, kid, N, bx, by, t)
    assert l1 < 0.1 * l0


def test_bf16_round_is_nearest_with_ties_to_even():
    """Against the definition: the nearest number with 8 significand bits (brute force over the
    two neighbours at the value's binade), ties to the one with an even last bit."""
    one = 1.0
    assert om.bf16_round(one) == one
    assert om.bf16_round(1 + 2.0 ** -8) == 1.0                    # tie, 1 is even
    assert om.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6      # tie, 1 + 2^-7 is odd
    assert om.bf16_round(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    assert om.bf16_round(-(1 + 2.0 ** -8 + 2.0 ** -20)) == -(1 + 2.0 ** -7)
    rng = np.random.default_rng(5)
    x = (rng.normal(size=20000) * 2.0 ** rng.integers(-20, 20, 20000)).astype(np.float32).astype(np.float64)
    m, e = np.frexp(np.abs(x))                                   # |x| = m 2^e, m in [0.5, 1)
    step = np.ldexp(1.0, e - 8)
    lo = np.floor(np.abs(x) / step) * step
    hi = lo + step
    dlo, dhi = np.abs(x) - lo, hi - np.abs(x)
    lo_even = (np.rint(lo / step) % 2) == 0
    want = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo_even, lo, hi))) * np.sign(x)
    assert np.array_equal(om.bf16_round(x), want)


def test_bf16_forward_equals_fp64_forward_on_representable_values():
    """With every weight and hidden value a bfloat16 number the rounded pass is the FP64 pass;
    a first-layer value off the bfloat16 grid moves the output by exactly its rounding."""
    p = {"W1": np.eye(4), "b1": np.zeros(4), "W2": np.eye(4), "b2": np.zeros(4),
         "w3": np.ones(4), "b3": np.array(0.5), "emb": np.array([0.25, -3.0])}
    args = (np.array([0, 1]), np.array([1 << 13, 1 << 26]), np.array([1 << 5, 1]), np.array([1 << 10, 1 << 5]))
    y, _ = om.forward(p, *args)
    assert np.array_equal(om.forward_bf16(p, *args), y)
    q = dict(p, b1=np.array([2.0 ** -9, 0.0, 0.0, 0.0]))            # h1[0] = 0.5 + 2^-9 -> 0.5
    yq, _ = om.forward(q, *args)
    assert np.allclose(yq - om.forward_bf16(q, *args), [2.0 ** -9, 2.0 ** -9], rtol=0, atol=1e-15)

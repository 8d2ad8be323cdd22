"""Pins of the FP64 reference of the ordering network (no GPU): finite differences, closed forms
of PAA, bfloat16 rounding against its bit-level definition, and an Adam step by hand."""
import numpy as np
import pytest

from oracle import mlp as M


def test_param_count():
    assert M.N_PARAMS == 32 * 256 + 256 + 256 * 256 + 256 + 256 + 1


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    theta = M.init_params(3) * 0.5
    theta += rng.normal(0, 0.01, theta.size)       # non-zero biases
    X = rng.normal(0, 1, (7, 32))
    t = rng.normal(0, 1, 7)
    _, g = M.loss_and_grads(theta, X, t)
    idx = np.concatenate([rng.integers(0, M.N_PARAMS, 40), [M.N_PARAMS - 1, 0, 32 * 256 + 3]])
    for k in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (M.loss_and_grads(tp, X, t)[0] - M.loss_and_grads(tm, X, t)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9), k


def test_forward_linear_region_closed_form():
    """With every pre-activation positive the network is affine: y = ((x W1 + b1) W2 + b2) w3 + b3."""
    rng = np.random.default_rng(2)
    p = {"W1": np.abs(rng.normal(0, 0.1, (32, 256))), "b1": np.full(256, 0.5),
         "W2": np.abs(rng.normal(0, 0.1, (256, 256))), "b2": np.full(256, 0.5),
         "w3": rng.normal(0, 0.1, 256), "b3": np.array([0.25])}
    X = np.abs(rng.normal(0, 1, (5, 32)))
    y, _ = M.forward(M.flatten(p), X)
    skip = np.log(((X[:, :16] - X[:, 16:]) ** 2).sum(axis=1) / 16 + 1e-4)
    want = ((X @ p["W1"] + p["b1"]) @ p["W2"] + p["b2"]) @ p["w3"] + 0.25 + skip
    np.testing.assert_allclose(y, want, rtol=1e-12)


def test_zero_output_layer_is_the_paa_distance():
    """With w3 = 0 and b3 = 0 the model's value is log(d / 16 + 1e-4) of the PAA distance d:
    identical halves give log(1e-4); halves that differ by 1 in one segment give log(1/16 + 1e-4);
    by 2 in every segment, d = 64 and the value is log(4 + 1e-4)."""
    theta = M.init_params(4)
    p = M.unflatten(theta)
    p["w3"] = np.zeros(256)
    p["b3"] = np.zeros(1)
    q = np.linspace(-1.5, 1.5, 16)
    X = np.stack([np.concatenate([q, q]), np.concatenate([q, q + np.eye(16)[5]]), np.concatenate([q, q - 2.0])])
    y, _ = M.forward(M.flatten(p), X)
    np.testing.assert_allclose(y, [np.log(1e-4), np.log(1 / 16 + 1e-4), np.log(4 + 1e-4)], rtol=1e-14)


def test_bf16_rounding_definition():
    # bfloat16 keeps 7 explicit mantissa bits: representable neighbours of 1 are 1 and 1 + 2^-7
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 2 ** -9, 1 + 3 * 2 ** -9, 1 + 3 * 2 ** -8, -3.14159, 1e-30, 0.0],
                    np.float32)
    got = M.bf16(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0                      # exact tie between 1 and 1 + 2^-7: to even (1)
    assert got[2] == 1.0                      # below the midpoint
    assert got[3] == 1 + 2 ** -7              # above the midpoint
    assert got[4] == 1 + 2 ** -6              # tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert got[5] == -3.140625
    assert got[7] == 0.0
    assert np.all((got.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_paa_closed_forms():
    x = np.arange(32, dtype=float)
    np.testing.assert_allclose(M.paa(x), np.arange(16) * 2 + 0.5)
    y = np.arange(20, dtype=float)     # uneven segments: boundaries floor(s*20/16)
    b = [(s * 20) // 16 for s in range(17)]
    np.testing.assert_allclose(M.paa(y), [y[b[s]:b[s + 1]].mean() for s in range(16)])
    assert M.paa(np.ones(100)).tolist() == [1.0] * 16


def test_adam_first_step_is_signed_lr():
    """At step 1 the bias-corrected update is lr * g / (|g| + eps) = lr * sign(g) for |g| >> eps."""
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -5.0, 1e-3])
    new, m, v = M.adam(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(new, theta - 0.01 * np.sign(g), rtol=1e-4)


def test_proposals_planted_copy_flat_series_and_tail():
    """Proposals: a planted affine copy of the query on the stride grid is proposed by its quarter
    at distance 0; the result is invariant to an affine change of the series; on a flat series
    every PAA is zero, so each quarter proposes its first start (lowest start on ties); quarters
    past the last candidate are empty."""
    from paper_1812_10302_amd import workloads as W
    rng = np.random.default_rng(11)
    T = W.random_walk(9000, 12).astype(np.float64)
    for m, p in ((128, 5002), (100, 3333), (300, 2048)):
        Q = 2.5 * T[p:p + m] - 7.0
        st, d = M.proposals(T, Q, block=1024)
        ps = m // 64 if m >= 128 else 1
        assert p % ps == 0
        k = p // 256
        assert st[k] == p and d[k] < 1e-20, (m, st[k], d[k])
        N = T.size - m + 1
        assert st.size == -(-N // 1024) * 4
        valid = st >= 0
        assert np.all(st[valid] // 256 == np.nonzero(valid)[0])
        assert np.all(st[valid] % ps == 0)
        np.testing.assert_array_equal(valid, np.arange(st.size) * 256 < N)
        st2, d2 = M.proposals(0.5 * T + 100.0, Q, block=1024)
        np.testing.assert_array_equal(st2, st)
        np.testing.assert_allclose(d2, d, rtol=1e-9, atol=1e-12)
    flat = np.full(3000, 4.0)
    Q = rng.normal(0, 1, 64)
    st, d = M.proposals(flat, Q, block=1024)
    N = flat.size - 64 + 1
    want = np.where(np.arange(st.size) * 256 < N, np.arange(st.size) * 256, -1)
    np.testing.assert_array_equal(st, want)
    assert np.allclose(d[st >= 0], (M.paa(np.asarray(Q - Q.mean()) / Q.std()) ** 2).sum())

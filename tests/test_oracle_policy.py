"""Pins of the attention-policy oracle (CPU only): the forward pass against
torch's float64 layers (layer_norm, linear, softmax attention with key
masking, tanh GELU), permutation invariance over the non-self tokens (the
property Sec. IV-B-1 builds on), and the inverse-CDF sampler."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

D, H, DH, F, L, NA = 64, 4, 16, 256, 2, 8


def _params(orc, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, orc.policy_num_params())
    return p


def _torch_policy(tokens, mask, th):
    t = torch.from_numpy(th)
    o = 0

    def take(*shape):
        nonlocal o
        n = int(np.prod(shape))
        v = t[o:o + n].view(*shape)
        o += n
        return v
    E, e = take(D, 6), take(D)
    x = torch.from_numpy(tokens)
    m = torch.from_numpy(mask.astype(bool))
    h = x @ E.T + e
    A, T = x.shape[0], x.shape[1]
    for _ in range(L):
        g1, b1n = take(D), take(D)
        Wqkv, bqkv = take(3 * D, D), take(3 * D)
        Wo, bo = take(D, D), take(D)
        g2, b2n = take(D), take(D)
        W1, b1 = take(F, D), take(F)
        W2, b2 = take(D, F), take(D)
        a = torch.nn.functional.layer_norm(h, (D,), g1, b1n, eps=1e-5)
        qkv = a @ Wqkv.T + bqkv
        q, k, v = qkv[..., :D], qkv[..., D:2 * D], qkv[..., 2 * D:]
        q = q.view(A, T, H, DH).transpose(1, 2)
        k = k.view(A, T, H, DH).transpose(1, 2)
        v = v.view(A, T, H, DH).transpose(1, 2)
        s = (q @ k.transpose(-1, -2)) / np.sqrt(DH)
        s = s.masked_fill(~m[:, None, None, :], float("-inf"))
        o_ = torch.softmax(s, -1) @ v
        o_ = o_.transpose(1, 2).reshape(A, T, D)
        h = h + o_ @ Wo.T + bo
        b = torch.nn.functional.layer_norm(h, (D,), g2, b2n, eps=1e-5)
        h = h + torch.nn.functional.gelu(b @ W1.T + b1, approximate="tanh") @ W2.T + b2
    gf, bf = take(D), take(D)
    Wh, bh = take(NA, D), take(NA)
    s0 = torch.nn.functional.layer_norm(h[:, 0], (D,), gf, bf, eps=1e-5)
    return (s0 @ Wh.T + bh).numpy()


def _tokens(A, n_agents, n_targets, seed, p_missing=0.2):
    rng = np.random.default_rng(seed)
    T = n_agents + n_targets
    x = np.zeros((A, T, 6))
    x[:, :, :2] = rng.normal(0, 3, (A, T, 2))
    x[:, 0, :3] = 0
    x[:, 0, 3] = 1
    x[:, 1:n_agents, 4] = 1
    x[:, n_agents:, 5] = 1
    mask = (rng.random((A, T)) > p_missing).astype(np.uint8)
    mask[:, 0] = 1
    x[..., :3] *= mask[..., None]
    return x, mask


def test_param_count(orc):
    per_layer = 2 * D + 3 * D * D + 3 * D + D * D + D + 2 * D + F * D + F + D * F + D
    assert orc.policy_num_params() == D * 6 + D + L * per_layer + 2 * D + NA * D + NA


def test_forward_matches_torch(orc):
    th = _params(orc, 1)
    x, mask = _tokens(30, 5, 5, 2)
    np.testing.assert_allclose(orc.policy_forward(x, mask, th), _torch_policy(x, mask, th),
                               rtol=1e-10, atol=1e-10)


def test_permutation_invariance_over_other_tokens(orc):
    th = _params(orc, 3)
    x, mask = _tokens(10, 5, 5, 4)
    base = orc.policy_forward(x, mask, th)
    rng = np.random.default_rng(5)
    perm = np.concatenate([[0], 1 + rng.permutation(9)])
    np.testing.assert_allclose(orc.policy_forward(x[:, perm], mask[:, perm], th), base,
                               rtol=1e-10, atol=1e-10)


def test_masked_tokens_do_not_matter(orc):
    th = _params(orc, 6)
    x, mask = _tokens(10, 3, 4, 7, p_missing=0.4)
    base = orc.policy_forward(x, mask, th)
    x2 = x.copy()
    x2[mask == 0, :2] = 123.0  # content of an excluded key is irrelevant for the self token
    np.testing.assert_allclose(orc.policy_forward(x2, mask, th)[:, :], base, rtol=1e-9, atol=1e-9)


def test_sampler_inverse_cdf(orc):
    lg = np.array([0.3, -1.0, 2.0, 0.0, 0.5, 9, 9, 9])
    p = np.exp(lg[:5] - lg[:5].max())
    p /= p.sum()
    c = np.cumsum(p)
    for u in [1e-6, c[0] - 1e-9, c[0] + 1e-9, 0.5, c[3] + 1e-9, 1 - 1e-9]:
        assert orc.policy_sample(lg, 5, u) == int(np.searchsorted(c, u, side="right"))
    from scipy import stats
    rng = np.random.default_rng(0)
    draws = [orc.policy_sample(lg, 5, u) for u in rng.random(20000)]
    assert stats.chisquare(np.bincount(draws, minlength=5), 20000 * p).pvalue > 1e-3

"""Pins of the attention-policy oracle (CPU only): the forward pass against
torch's float64 layers (layer_norm, linear, softmax attention with key
masking, tanh GELU), permutation invariance over the non-self tokens (the
property Sec. IV-B-1 builds on), the inverse-CDF sampler, and the recurrent
form of Fig. 3 (a carried state as an extra first row): against torch, its
reduction to the plain form when the state is an embedded token, the head
on the returned state, and invariance to any order of the tokens. The
backward pass: central differences of the forward pass in sampled entries of
every parameter group, and the whole gradient against torch's float64
autograd of the torch network (plain and recurrent forms, masked keys)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

D, H, DH, F, L, NA = 64, 4, 16, 256, 2, 8


def _params(orc, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, orc.policy_num_params())
    return p


def _torch_policy(tokens, mask, th, hidden=None):
    t = th if isinstance(th, torch.Tensor) else torch.from_numpy(th)
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
    if hidden is not None:  # the recurrent row ahead of the embedded tokens, never masked
        hid = hidden if isinstance(hidden, torch.Tensor) else torch.from_numpy(hidden)
        h = torch.cat([hid[:, None], h], 1)
        m = torch.cat([torch.ones_like(m[:, :1]), m], 1)
    A, T = h.shape[0], h.shape[1]
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
    out = s0 @ Wh.T + bh
    return out if isinstance(th, torch.Tensor) else out.numpy()


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


def test_recurrent_form_matches_torch(orc):
    th = _params(orc, 5)
    x, mask = _tokens(7, 3, 2, seed=8)
    rng = np.random.default_rng(3)
    hid = rng.normal(0, 1.0, (7, D))
    lg, hout = orc.policy_forward_rec(x, mask, hid, th)
    np.testing.assert_allclose(lg, _torch_policy(x, mask, th, hid), atol=1e-10)
    # no state: zeros
    lz, _ = orc.policy_forward_rec(x, mask, None, th)
    np.testing.assert_allclose(lz, _torch_policy(x, mask, th, np.zeros((7, D))), atol=1e-10)


def test_recurrent_form_reduces_to_plain_form(orc):
    # a carried state equal to the embedding of a token x0 is that token put first
    th = _params(orc, 6)
    x, mask = _tokens(5, 2, 3, seed=9)
    x0 = np.random.default_rng(4).normal(0, 1.0, (5, 6))
    E, e = th[:D * 6].reshape(D, 6), th[D * 6:D * 7]
    lg, _ = orc.policy_forward_rec(x, mask, x0 @ E.T + e, th)
    full = np.concatenate([x0[:, None], x], 1)
    fm = np.concatenate([np.ones((5, 1), np.uint8), mask], 1)
    np.testing.assert_allclose(lg, orc.policy_forward(full, fm, th), atol=1e-12)


def test_recurrent_state_is_the_heads_input(orc):
    th = _params(orc, 7)
    x, mask = _tokens(4, 2, 2, seed=10)
    hid = np.random.default_rng(5).normal(0, 1.0, (4, D))
    lg, hout = orc.policy_forward_rec(x, mask, hid, th)
    n = th.size
    Wh, bh = th[n - NA * D - NA:n - NA].reshape(NA, D), th[n - NA:]
    np.testing.assert_allclose(lg, hout @ Wh.T + bh, atol=1e-12)
    # the state is a final LayerNorm output: (s - beta) / gamma has mean 0, variance ~1
    gf, bf = th[n - NA * D - NA - 2 * D:n - NA * D - NA - D], th[n - NA * D - NA - D:n - NA * D - NA]
    z = (hout - bf) / gf
    np.testing.assert_allclose(z.mean(1), 0.0, atol=1e-10)
    assert np.all(np.abs(z.var(1) - 1.0) < 1e-3)
    # two steps: the second sees the first's state
    lg2, h2 = orc.policy_forward_rec(x, mask, hout, th)
    np.testing.assert_allclose(lg2, _torch_policy(x, mask, th, hout), atol=1e-10)
    assert np.abs(h2 - hout).max() > 1e-3


def test_recurrent_form_ignores_token_order(orc):
    th = _params(orc, 8)
    x, mask = _tokens(3, 3, 3, seed=11)
    hid = np.random.default_rng(6).normal(0, 1.0, (3, D))
    lg, hout = orc.policy_forward_rec(x, mask, hid, th)
    perm = np.random.default_rng(7).permutation(x.shape[1])
    lp, hp = orc.policy_forward_rec(x[:, perm], mask[:, perm], hid, th)
    np.testing.assert_allclose(lp, lg, atol=1e-12)
    np.testing.assert_allclose(hp, hout, atol=1e-12)


PER_LAYER = 2 * D + 3 * D * D + 3 * D + D * D + D + 2 * D + F * D + F + D * F + D
GROUPS = [("E", D * 6), ("e", D)] + [
    (f"{n}{l}", s) for l in range(L) for n, s in (
        ("ln1g", D), ("ln1b", D), ("Wq", D * D), ("Wk", D * D), ("Wv", D * D), ("bqkv", 3 * D),
        ("Wo", D * D), ("bo", D), ("ln2g", D), ("ln2b", D), ("W1", F * D), ("b1", F),
        ("W2", D * F), ("b2", D))] + [("lnfg", D), ("lnfb", D), ("Wh", NA * D), ("bh", NA)]


def test_backward_matches_central_differences(orc):
    th = _params(orc, 11)
    x, mask = _tokens(3, 2, 3, seed=12)
    dl = np.random.default_rng(13).normal(size=(3, NA))
    g = orc.policy_backward(x, mask, th, dl)
    assert sum(s for _, s in GROUPS) == th.size
    rng = np.random.default_rng(14)
    off, h = 0, 1e-5
    for name, size in GROUPS:
        for i in off + rng.choice(size, min(size, 4), replace=False):
            tp, tm = th.copy(), th.copy()
            tp[i] += h
            tm[i] -= h
            fd = ((orc.policy_forward(x, mask, tp) - orc.policy_forward(x, mask, tm)) * dl).sum()
            assert g[i] == pytest.approx(fd / (2 * h), abs=1e-8 * max(1.0, np.abs(g).max())), name
        off += size


def test_backward_matches_autograd(orc):
    th = _params(orc, 15)
    x, mask = _tokens(4, 3, 2, seed=16)
    dl = np.random.default_rng(17).normal(size=(4, NA))
    t = torch.tensor(th, requires_grad=True)
    (_torch_policy(x, mask, t) * torch.from_numpy(dl)).sum().backward()
    np.testing.assert_allclose(orc.policy_backward(x, mask, th, dl), t.grad.numpy(), rtol=0,
                               atol=1e-11 * np.abs(t.grad.numpy()).max())


def test_recurrent_backward_matches_autograd(orc):
    th = _params(orc, 18)
    x, mask = _tokens(3, 2, 2, seed=19)
    rng = np.random.default_rng(20)
    hid = rng.normal(0, 1.0, (3, D))
    dl = rng.normal(size=(3, NA))
    t = torch.tensor(th, requires_grad=True)
    hv = torch.tensor(hid, requires_grad=True)
    (_torch_policy(x, mask, t, hv) * torch.from_numpy(dl)).sum().backward()
    g, dh = orc.policy_backward_rec(x, mask, hid, th, dl)
    np.testing.assert_allclose(g, t.grad.numpy(), rtol=0, atol=1e-11 * np.abs(g).max())
    np.testing.assert_allclose(dh, hv.grad.numpy(), rtol=0, atol=1e-11 * np.abs(dh).max())
    # no state: zeros, and the embedding takes no gradient from the state row
    g0, _ = orc.policy_backward_rec(x, mask, None, th, dl)
    g1, _ = orc.policy_backward_rec(x, mask, np.zeros((3, D)), th, dl)
    np.testing.assert_array_equal(g0, g1)


def _chain_loss_torch(xs, ms, t, dls):
    h = torch.zeros(xs[0].shape[0], D, dtype=torch.float64)
    loss = 0.0
    for x, m, dl in zip(xs, ms, dls):
        out, h = _torch_policy_rec(x, m, t, h)
        loss = loss + (out * torch.from_numpy(dl)).sum()
    return loss


def _torch_policy_rec(x, m, t, h):
    """Torch form of one recurrent step: (logits, next state)."""
    return _torch_policy(x, m, t, h), _torch_state(x, m, t, h)


def _torch_state(x, m, t, h):
    """LN_f of the carried row after the trunk (the next state), torch float64."""
    o = 0

    def take(*shape):
        nonlocal o
        k = int(np.prod(shape))
        v = t[o:o + k].view(*shape)
        o += k
        return v
    E, e = take(D, 6), take(D)
    xx = torch.from_numpy(x)
    mm = torch.from_numpy(m.astype(bool))
    hh = torch.cat([h[:, None], xx @ E.T + e], 1)
    mm = torch.cat([torch.ones_like(mm[:, :1]), mm], 1)
    A_, T_ = hh.shape[0], hh.shape[1]
    for _ in range(L):
        g1, b1n = take(D), take(D)
        Wqkv, bqkv = take(3 * D, D), take(3 * D)
        Wo, bo = take(D, D), take(D)
        g2, b2n = take(D), take(D)
        W1, b1 = take(F, D), take(F)
        W2, b2 = take(D, F), take(D)
        a = torch.nn.functional.layer_norm(hh, (D,), g1, b1n, eps=1e-5)
        qkv = a @ Wqkv.T + bqkv
        q, k, v = qkv[..., :D], qkv[..., D:2 * D], qkv[..., 2 * D:]
        q = q.view(A_, T_, H, DH).transpose(1, 2)
        k = k.view(A_, T_, H, DH).transpose(1, 2)
        v = v.view(A_, T_, H, DH).transpose(1, 2)
        s = (q @ k.transpose(-1, -2)) / np.sqrt(DH)
        s = s.masked_fill(~mm[:, None, None, :], float("-inf"))
        o_ = (torch.softmax(s, -1) @ v).transpose(1, 2).reshape(A_, T_, D)
        hh = hh + o_ @ Wo.T + bo
        b = torch.nn.functional.layer_norm(hh, (D,), g2, b2n, eps=1e-5)
        hh = hh + torch.nn.functional.gelu(b @ W1.T + b1, approximate="tanh") @ W2.T + b2
    gf, bf = take(D), take(D)
    return torch.nn.functional.layer_norm(hh[:, 0], (D,), gf, bf, eps=1e-5)


def test_bptt_matches_autograd_through_the_sequence(orc):
    # three recurrent steps from zeros: the chained oracle gradient against
    # torch float64 autograd through the whole sequence
    th = _params(orc, 21)
    rng = np.random.default_rng(22)
    T_, A_ = 3, 4
    xs, ms = zip(*[_tokens(A_, 2, 2, seed=30 + s) for s in range(T_)])
    dls = [rng.normal(size=(A_, NA)) for _ in range(T_)]
    t = torch.tensor(th, requires_grad=True)
    _chain_loss_torch(xs, ms, t, dls).backward()
    g = orc.policy_bptt(np.stack(xs), np.stack(ms), th, np.stack(dls))
    np.testing.assert_allclose(g, t.grad.numpy(), rtol=0, atol=1e-10 * np.abs(g).max())
    # one-step gradients (each step's state taken as a constant input) miss the
    # later steps' dependence on the state
    states, h = [], None
    for s in range(T_):
        states.append(h)
        h = orc.policy_forward_rec(xs[s], ms[s], h, th)[1]
    g1 = sum(orc.policy_backward_rec(xs[s], ms[s], states[s], th, dls[s])[0] for s in range(T_))
    assert np.abs(g1 - g).max() > 1e-3 * np.abs(g).max()


def test_bptt_matches_central_differences(orc):
    th = _params(orc, 23)
    rng = np.random.default_rng(24)
    xs, ms = zip(*[_tokens(2, 2, 1, seed=40 + s) for s in range(3)])
    dls = np.stack([rng.normal(size=(2, NA)) for _ in range(3)])

    def loss(p):
        h, tot = None, 0.0
        for s in range(3):
            lg, h = orc.policy_forward_rec(xs[s], ms[s], h, p)
            tot += (lg * dls[s]).sum()
        return tot
    g = orc.policy_bptt(np.stack(xs), np.stack(ms), th, dls)
    for i in rng.choice(th.size, 12, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[i] += 1e-5
        tm[i] -= 1e-5
        assert g[i] == pytest.approx((loss(tp) - loss(tm)) / 2e-5, abs=1e-8 * max(1.0, np.abs(g).max()))

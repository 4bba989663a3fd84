"""FP64 CPU oracle of the learner's forward half: the centralised critic's
inputs, generalised advantage estimation, the clipped PPO objective and the
gradient of a network's output head.

TEST INFRASTRUCTURE ONLY: plain numpy loops, written for reading against the
definitions; only the tests, the package's smoke check and the benchmark's
CPU-baseline leg may call it. It shares nothing with the HIP library.

Paper: MAPPO (Sec. III-B): each agent's actor is updated with the PPO clipped
surrogate objective and one centralised critic estimates V(S) from the global
state; TransfMAPPO (Sec. IV-B-1, Fig. 3): the critic is a transformer over
the global state's entity tokens with an extra embedding token whose
transformed output gives V(s). Readings (the paper is silent on them): the
advantage is GAE(gamma, lambda) (Schulman et al. 2016) of the env's shared
reward under V, one per env-step and shared by the env's agents; a step with
done = 1 does not bootstrap; the value target is A + V; the value loss is the
plain squared error; the critic's entity token of an agent or target is
(x / s, y / s, v cos(psi), v sin(psi), is_agent, is_target) with s a position
scale, and its extra token is all zeros (its embedding is the embedding bias).
"""
import numpy as np


def critic_tokens(gstate, n_agents: int, n_targets: int, pos_scale: float):
    """gstate [N][n_agents + n_targets][6] rows (x, y, z, speed, heading,
    is_target) of N env-states -> tokens [N][1 + n_agents + n_targets][6]:
    the value token (zeros), then every agent and target in order."""
    g = np.asarray(gstate, np.float64)
    N, M, _ = g.shape
    assert M == n_agents + n_targets
    tok = np.zeros((N, 1 + M, 6))
    for n in range(N):
        for k in range(M):
            x, y, _, v, psi, is_t = g[n, k]
            tok[n, 1 + k] = (x / pos_scale, y / pos_scale, v * np.cos(psi), v * np.sin(psi),
                             1.0 - is_t, is_t)
    return tok


def gae(rewards, dones, values, gamma: float, lam: float):
    """rewards, dones [T][E]; values [T + 1][E] (V of the state before step
    t, and after the last step) -> (advantages [T][E], returns [T][E]):
    delta_t = r_t + gamma V_{t+1} (1 - d_t) - V_t,
    A_t = delta_t + gamma lambda (1 - d_t) A_{t+1}, R_t = A_t + V_t."""
    r = np.asarray(rewards, np.float64)
    d = np.asarray(dones, np.float64)
    v = np.asarray(values, np.float64)
    T, E = r.shape
    adv = np.zeros((T, E))
    for e in range(E):
        nxt = 0.0
        for t in range(T - 1, -1, -1):
            cont = 1.0 - d[t, e]
            delta = r[t, e] + gamma * v[t + 1, e] * cont - v[t, e]
            nxt = delta + gamma * lam * cont * nxt
            adv[t, e] = nxt
    return adv, adv + v[:T]


def _log_softmax(z):
    m = z.max()
    return z - m - np.log(np.exp(z - m).sum())


def ppo_objective(logits_new, logits_old, actions, adv, values, returns, n_agents: int,
                  n_actions: int, clip_eps: float):
    """Samples: (step t, agent a), agent a of env a // n_agents.
    logits_* [T][A][>= n_actions] (the first n_actions are the action
    logits), actions [T][A], adv [T][E], values / returns [T][E].
    Returns dict: policy_loss = -mean min(rho A, clip(rho, 1 - eps, 1 + eps) A)
    with rho = pi_new(a) / pi_old(a); value_loss = mean (V - R)^2;
    entropy = mean H(pi_new); clip_frac = share of samples whose clipped term
    is strictly the smaller; dlogits [T][A][n_actions] = d policy_loss / d
    logits_new; dvalues [T][E] = d value_loss / d V."""
    ln = np.asarray(logits_new, np.float64)
    lo = np.asarray(logits_old, np.float64)
    act = np.asarray(actions)
    T, A = act.shape
    E = A // n_agents
    N = T * A
    pl = ent = 0.0
    clipped = 0
    dlog = np.zeros((T, A, n_actions))
    for t in range(T):
        for a in range(A):
            e = a // n_agents
            lpn = _log_softmax(ln[t, a, :n_actions])
            lpo = _log_softmax(lo[t, a, :n_actions])
            k = int(act[t, a])
            rho = np.exp(lpn[k] - lpo[k])
            A_ = adv[t, e]
            unc = rho * A_
            clp = min(max(rho, 1.0 - clip_eps), 1.0 + clip_eps) * A_
            p = np.exp(lpn)
            ent += -(p * lpn).sum()
            if clp < unc:  # the clipped term is the minimum: no gradient
                pl += clp
                clipped += 1
            else:
                pl += unc
                onehot = np.zeros(n_actions)
                onehot[k] = 1.0
                # d(rho)/d logits = rho (onehot - p); the loss is -mean(...)
                dlog[t, a] = -(A_ * rho) * (onehot - p) / N
    v = np.asarray(values, np.float64)
    R = np.asarray(returns, np.float64)
    return {
        "policy_loss": -pl / N,
        "value_loss": float(((v - R) ** 2).mean()),
        "entropy": ent / N,
        "clip_frac": clipped / N,
        "dlogits": dlog,
        "dvalues": 2.0 * (v - R) / v.size,
    }


def head_grad(feat, dout, n_out: int, rows: int = 8):
    """Gradient of the linear output head y = W f + b (W [rows][64], b [rows])
    from the gradients at its outputs: feat [N][64] the head's inputs,
    dout [N][>= n_out] d loss / d y for the first n_out outputs (the others
    take no gradient). Returns (dW [rows][64], db [rows]) with
    dW[k][d] = sum_n dout[n][k] f[n][d], db[k] = sum_n dout[n][k]."""
    f = np.asarray(feat, np.float64)
    g = np.asarray(dout, np.float64).reshape(f.shape[0], -1)[:, :n_out]
    dW = np.zeros((rows, f.shape[1]))
    db = np.zeros(rows)
    dW[:n_out] = g.T @ f
    db[:n_out] = g.sum(0)
    return dW, db

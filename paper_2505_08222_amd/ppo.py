"""The learner (argument marshalling only): critic values of global states,
generalised advantage estimation, the clipped PPO objective, the gradient
and Adam update of the output heads, and the networks' training form (an
FP32 forward pass with its tape and the exact reverse pass into every
parameter) for the full update (MAPPO, Sec. III-B; TransfMAPPO, Sec. IV-B-1,
Fig. 3). Every step runs in the HIP library."""
import ctypes as C

import torch

from ._lib import check, lib, ptr


def _l():
    L = lib()
    if not getattr(L, "_ppo_registered", False):
        V, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        L.critic_workspace_bytes.argtypes = [I64, I32, I32]
        L.critic_workspace_bytes.restype = I64
        L.critic_forward.argtypes = [V, I64, I32, I32, F, V, V, V, V, I64, V]
        L.critic_forward.restype = C.c_int
        L.ppo_gae.argtypes = [V, V, V, I32, I64, F, F, V, V, V]
        L.ppo_gae.restype = C.c_int
        L.ppo_workspace_bytes.argtypes = []
        L.ppo_workspace_bytes.restype = I64
        L.ppo_objective.argtypes = [V, V, V, V, V, V, I32, I64, I32, I32, F, V, V, V, V, I64, V]
        L.ppo_objective.restype = C.c_int
        L.head_grad.argtypes = [I64, V, V, I32, I32, V, V, I64, V]
        L.head_grad.restype = C.c_int
        L.policy_forward_feat.argtypes = [I64, I32, I32, I32, V, V, V, V, V, V, C.c_uint64,
                                          C.c_uint32, C.c_uint32, V, I64, V]
        L.policy_forward_feat.restype = C.c_int
        L.critic_forward_rec.argtypes = [V, I32, I64, I32, I32, F, V, V, V, V, V, I64, V]
        L.critic_forward_rec.restype = C.c_int
        L.policy_train_workspace_bytes.argtypes = [I64, I32]
        L.policy_train_workspace_bytes.restype = I64
        L.policy_train_forward.argtypes = [I64, I32, I32, V, V, V, V, V, V, V, I64, V]
        L.policy_train_forward.restype = C.c_int
        L.critic_train_forward.argtypes = [V, I64, I32, I32, F, I32, V, V, V, V, V, I64, V]
        L.critic_train_forward.restype = C.c_int
        L.policy_train_backward.argtypes = [I64, I32, I32, V, V, I32, I32, V, I32, V, V, V, I64,
                                            V]
        L.policy_train_backward.restype = C.c_int
        L._ppo_registered = True
    return L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


HEAD_PARAMS = 8 * 64 + 8  # the head: the last floats of the parameter vector


def critic_forward(gstate, n_agents: int, n_targets: int, params, pos_scale: float = 1000.0,
                   features: bool = False):
    """gstate [N, n_agents + n_targets, 6] (or the rollout's [T, E*M, 6]) ->
    values [N] (and the head's input features [N, 64] with features=True)."""
    M = n_agents + n_targets
    g = gstate.reshape(-1, M, 6).contiguous()
    N = g.shape[0]
    L = _l()
    n = L.critic_workspace_bytes(N, n_agents, n_targets)
    buf = torch.empty(n + 256, dtype=torch.uint8, device=g.device)
    w = (buf.data_ptr() + 255) & ~255
    out = torch.empty(N, dtype=torch.float32, device=g.device)
    feat = torch.empty((N, 64), dtype=torch.float32, device=g.device) if features else None
    check(L.critic_forward(ptr(g), N, n_agents, n_targets, pos_scale, ptr(params), ptr(out),
                           ptr(feat), C.c_void_p(w), n, _stream()))
    return (out, feat) if features else out


def critic_forward_rec(gstate, n_agents: int, n_targets: int, params, hidden=None,
                       pos_scale: float = 1000.0):
    """The recurrent critic over a trajectory: gstate [T, N, n_agents +
    n_targets, 6] (or the rollout's [T, N * M, 6]), hidden [N, 64] or None
    (zeros) -> (values [T, N], states [T, N, 64]; states[t] is the head's
    input at step t and the state carried into step t + 1)."""
    M = n_agents + n_targets
    T = gstate.shape[0]
    g = gstate.reshape(T, -1, M, 6).contiguous()
    N = g.shape[1]
    L = _l()
    n = L.critic_workspace_bytes(N, n_agents, n_targets)
    buf = torch.empty(n + 256, dtype=torch.uint8, device=g.device)
    w = (buf.data_ptr() + 255) & ~255
    values = torch.empty((T, N), dtype=torch.float32, device=g.device)
    states = torch.empty((T, N, 64), dtype=torch.float32, device=g.device)
    check(L.critic_forward_rec(ptr(g), T, N, n_agents, n_targets, pos_scale, ptr(params),
                               ptr(hidden), ptr(values), ptr(states), C.c_void_p(w), n, _stream()))
    return values, states


def policy_features(obs, mask, params, n_tok: int, n_agents: int, n_actions: int = 5):
    """obs [A * n_tok, 6], mask [A * n_tok] -> (logits [A, 8], features [A, 64])."""
    from .policy import _work
    A = obs.shape[0] // n_tok
    logits = torch.empty((A, 8), dtype=torch.float32, device=obs.device)
    feat = torch.empty((A, 64), dtype=torch.float32, device=obs.device)
    buf, w, n = _work(A, A * n_tok, obs.device)
    check(_l().policy_forward_feat(A, n_tok, n_agents, n_actions, ptr(obs.contiguous()),
                                   ptr(mask.contiguous()), ptr(params), ptr(logits), None,
                                   ptr(feat), C.c_uint64(0), 0, 0, w, n, _stream()))
    del buf
    return logits, feat


def head_grad(feat, dout, n_out: int):
    """feat [N, 64], dout [N, ld] (or [N] for one output) -> the head's
    gradient [520] (Wh [8, 64], bh [8])."""
    N = feat.shape[0]
    d = (dout.reshape(N, 1) if dout.dim() == 1 else dout.reshape(N, dout.shape[-1])).contiguous()
    L = _l()
    work = torch.empty(L.ppo_workspace_bytes(), dtype=torch.uint8, device=feat.device)
    g = torch.empty(HEAD_PARAMS, dtype=torch.float32, device=feat.device)
    check(L.head_grad(N, ptr(feat.contiguous()), ptr(d), d.shape[1], n_out, ptr(g), ptr(work),
                      work.numel(), _stream()))
    return g


def gae(rewards, dones, values, gamma: float, lam: float):
    """rewards [T, E], dones [T, E] (uint8), values [T + 1, E] -> (adv, ret)."""
    T, E = rewards.shape
    adv = torch.empty_like(rewards)
    ret = torch.empty_like(rewards)
    check(_l().ppo_gae(ptr(rewards.contiguous()), ptr(dones.contiguous()), ptr(values.contiguous()),
                       T, E, gamma, lam, ptr(adv), ptr(ret), _stream()))
    return adv, ret


def objective(logits_new, logits_old, actions, adv, values, returns, n_agents: int,
              n_actions: int, clip_eps: float = 0.2, grads: bool = True):
    """logits [T, A, 8], actions [T, A], adv / values / returns [T, E] ->
    (out [4] float64: policy loss, value loss, entropy, clip fraction;
    dlogits [T, A, 8] or None; dvalues [T, E] or None)."""
    T, A = actions.shape
    L = _l()
    work = torch.empty(L.ppo_workspace_bytes(), dtype=torch.uint8, device=actions.device)
    out = torch.empty(4, dtype=torch.float64, device=actions.device)
    dl = torch.empty_like(logits_new) if grads else None
    dv = torch.empty_like(values) if grads else None
    check(L.ppo_objective(ptr(logits_new.contiguous()), ptr(logits_old.contiguous()),
                          ptr(actions.contiguous()), ptr(adv.contiguous()), ptr(values.contiguous()),
                          ptr(returns.contiguous()), T, A, n_agents, n_actions, clip_eps, ptr(out),
                          ptr(dl), ptr(dv), ptr(work), work.numel(), _stream()))
    return out, dl, dv


class HeadAdam:
    """Adam state of one network's output head (the last HEAD_PARAMS floats
    of its parameter vector); step() updates them in place on the device."""

    def __init__(self, params, lr=3e-4, betas=(0.9, 0.999), eps=1e-8):
        self.params = params
        self.head = params[params.numel() - HEAD_PARAMS:]
        self.m = torch.zeros_like(self.head)
        self.v = torch.zeros_like(self.head)
        self.lr, (self.b1, self.b2), self.eps = float(lr), betas, float(eps)
        self.step_count = 0

    def step(self, grad):
        self.step_count += 1
        check(lib().mlp_adam_step(HEAD_PARAMS, ptr(self.head), ptr(grad), ptr(self.m), ptr(self.v),
                                  self.lr, self.b1, self.b2, self.eps, self.step_count, _stream()))


class TrainPass:
    """Workspace and calls of the training form for batches of A agents (or
    critic states) with n_tok rows each (rec = 1: the recurrent form, the
    carried state first). forward() records the tape that backward() reads."""

    def __init__(self, A: int, n_tok: int, rec: int = 0, device="cuda"):
        L = _l()
        self.A, self.n_tok, self.rec = int(A), int(n_tok), int(rec)
        n = int(L.policy_train_workspace_bytes(self.A, self.n_tok))
        assert n > 0, "bad sizes"
        self._buf = torch.empty(n + 256, dtype=torch.uint8, device=device)
        off = (-self._buf.data_ptr()) % 256
        self._w, self._n = C.c_void_p(self._buf.data_ptr() + off), n
        self.device = device

    def forward(self, obs, mask, params, hidden=None):
        """obs [A * (n_tok - rec), 6], mask -> (logits [A, 8], features [A, 64])."""
        logits = torch.empty((self.A, 8), dtype=torch.float32, device=self.device)
        feat = torch.empty((self.A, 64), dtype=torch.float32, device=self.device)
        check(_l().policy_train_forward(self.A, self.n_tok, self.rec, ptr(obs.contiguous()),
                                        ptr(mask.contiguous()), ptr(hidden), ptr(params),
                                        ptr(logits), ptr(feat), self._w, self._n, _stream()))
        return logits, feat

    def critic_forward(self, gstate, n_agents: int, n_targets: int, params, hidden=None,
                       pos_scale: float = 1000.0):
        """gstate [A, n_agents + n_targets, 6] -> (values [A], features [A, 64])."""
        assert self.n_tok == n_agents + n_targets + 1
        g = gstate.reshape(self.A, n_agents + n_targets, 6).contiguous()
        values = torch.empty(self.A, dtype=torch.float32, device=self.device)
        feat = torch.empty((self.A, 64), dtype=torch.float32, device=self.device)
        check(_l().critic_train_forward(ptr(g), self.A, n_agents, n_targets, pos_scale, self.rec,
                                        ptr(hidden), ptr(params), ptr(values), ptr(feat), self._w,
                                        self._n, _stream()))
        return values, feat

    def backward(self, params, dout, n_out: int, grad=None, dnext=None, accumulate=False):
        """dout [A, ld] (or [A]), dnext [A, 64] (the gradient at the state
        passed on, or None) -> (gradient [P] (added to `grad` with
        accumulate), gradient at the carried state [A, 64] or None)."""
        d = (dout.reshape(self.A, 1) if dout.dim() == 1
             else dout.reshape(self.A, dout.shape[-1])).contiguous()
        if grad is None:
            grad = torch.empty_like(params)
            accumulate = False
        dh = (torch.empty((self.A, 64), dtype=torch.float32, device=self.device)
              if self.rec else None)
        dn = None if dnext is None else dnext.contiguous()
        check(_l().policy_train_backward(self.A, self.n_tok, self.rec, ptr(params), ptr(d),
                                         d.shape[1], n_out, ptr(dn), int(bool(accumulate)),
                                         ptr(grad), ptr(dh), self._w, self._n, _stream()))
        return grad, dh


def chain_forward(tp: TrainPass, forward, T: int):
    """The forward chain of T steps of the recurrent form from zeros:
    forward(t, hidden) runs step t's training-form forward pass on `tp`
    (tp.forward or tp.critic_forward with the step's inputs) and returns its
    outputs, the second being the state it passes on. Returns (first outputs
    [T, ...], states [T, A, 64])."""
    assert tp.rec == 1
    outs, states = [], []
    h = None
    for t in range(T):
        o = forward(t, h)
        outs.append(o[0].clone())
        h = o[1].clone()
        states.append(h)
    return torch.stack(outs), torch.stack(states)


def chain_backward(tp: TrainPass, forward, states, douts, params, n_out: int, grad=None):
    """The reverse pass of a chain recorded by chain_forward: the steps in
    reverse order, each forward pass taken again from its input state and
    reversed with the following step's state gradient, the parameter
    gradients summed. douts[t]: the loss gradient at step t's outputs."""
    T = len(douts)
    dnext = None
    for t in range(T - 1, -1, -1):
        forward(t, states[t - 1] if t > 0 else None)
        grad, dnext = tp.backward(params, douts[t], n_out, grad=grad, dnext=dnext,
                                  accumulate=t < T - 1)
    return grad


def bptt(tp: TrainPass, forward, douts, params, n_out: int, grad=None):
    """Back-propagation through time over T = len(douts) steps of the
    recurrent form started from zeros (chain_forward, then chain_backward).
    Returns (gradient [P], the states [T, A, 64])."""
    _, states = chain_forward(tp, forward, len(douts))
    return chain_backward(tp, forward, states, douts, params, n_out, grad), states


class Learner:
    """The learner's loop over one batch of closed-loop experience (MAPPO,
    Sec. III-B, with the TransfMAPPO networks): critic values of every
    state, GAE, then `epochs` passes over `minibatches` groups, each a
    training-form forward and reverse pass of the actor (clipped surrogate)
    and the critic (squared error to the GAE returns) and an Adam step on
    every parameter of both. Plain form: minibatches of whole steps.
    Recurrent form (recurrent=True, both networks with their carried
    state, started from zeros at the batch's first step, an episode start):
    minibatches of whole envs over all steps, differentiated through time.
    Orchestration only: every step of it is one of the library's entry
    points."""

    def __init__(self, actor, critic, n_agents: int, n_targets: int, n_actions: int = 5,
                 lr: float = 3e-4, clip_eps: float = 0.2, gamma: float = 0.99, lam: float = 0.95,
                 pos_scale: float = 1000.0, recurrent: bool = False, behaviour: str = "inference"):
        from .learned import Adam
        self.recurrent = bool(recurrent)
        # the old policy's logits and the values for GAE: "inference" takes the
        # inference kernels (BF16; the old logits are then exactly those of the
        # policy that sampled the closed loop's actions), "training" the FP32
        # training form (then the first ratio is exactly 1)
        assert behaviour in ("inference", "training")
        self.behaviour = behaviour
        self.actor, self.critic = actor, critic
        self.na, self.nt, self.n_actions = n_agents, n_targets, n_actions
        self.opt_a, self.opt_c = Adam(actor, lr=lr), Adam(critic, lr=lr)
        self.clip_eps, self.gamma, self.lam, self.pos_scale = clip_eps, gamma, lam, pos_scale
        self._passes = {}

    def _pass(self, A, n_tok, rec=0):
        key = (A, n_tok, rec)
        if key not in self._passes:
            self._passes[key] = TrainPass(A, n_tok, rec, device=self.actor.device)
        return self._passes[key]

    def _critic_fn(self, tp, gs):
        return lambda t, h: tp.critic_forward(gs[t], self.na, self.nt, self.critic, hidden=h,
                                              pos_scale=self.pos_scale)

    def _actor_fn(self, tp, obs, mask):
        return lambda t, h: tp.forward(obs[t], mask[t], self.actor, h)

    def values(self, gstate):
        """V of states gstate [S, E, M, 6] -> [S, E] (training form, FP32;
        the recurrent critic runs them in order from zeros)."""
        S = gstate.shape[0]
        M = self.na + self.nt
        gs = gstate.reshape(S, -1, M, 6)
        E = gs.shape[1]
        tp = self._pass(E, M + 1, int(self.recurrent))
        if self.recurrent:
            return chain_forward(tp, self._critic_fn(tp, gs), S)[0]
        return torch.stack([tp.critic_forward(gs[s], self.na, self.nt, self.critic,
                                              pos_scale=self.pos_scale)[0].clone()
                            for s in range(S)])

    def logits(self, obs, mask):
        """Actor logits of obs [T, A * n_tok, 6] -> [T, A, 8] (training form;
        the recurrent actor runs the steps in order from zeros)."""
        T = obs.shape[0]
        n_tok = self.na + self.nt
        A = obs.shape[1] // n_tok
        if self.recurrent:
            tp = self._pass(A, n_tok + 1, 1)
            return chain_forward(tp, self._actor_fn(tp, obs, mask), T)[0]
        tp = self._pass(A, n_tok)
        return torch.stack([tp.forward(obs[t], mask[t], self.actor)[0].clone() for t in range(T)])

    def _behaviour(self, obs, mask, gs):
        """Values [T + 1, E] and old logits [T, A, 8] from the inference
        kernels: the critic over every state in one call (in order through
        its carried state when recurrent), the actor step by step."""
        from . import policy
        S, E = gs.shape[0], gs.shape[1]
        T = obs.shape[0]
        n_tok = self.na + self.nt
        A = obs.shape[1] // n_tok
        if self.recurrent:
            values = critic_forward_rec(gs, self.na, self.nt, self.critic,
                                        pos_scale=self.pos_scale)[0]
            h = None
            logits = []
            for t in range(T):
                lg, _, h = policy.forward_rec(obs[t], mask[t], h, self.actor, n_tok, self.na,
                                              self.n_actions)
                logits.append(lg)
            return values, torch.stack(logits)
        values = critic_forward(gs.reshape(S * E, self.na + self.nt, 6), self.na, self.nt,
                                self.critic, pos_scale=self.pos_scale).reshape(S, E)
        logits = torch.stack([policy.forward(obs[t], mask[t], self.actor, n_tok, self.na,
                                             self.n_actions)[0] for t in range(T)])
        return values, logits.reshape(T, A, 8)

    def update(self, obs, mask, actions, gstate, rewards, dones, epochs: int = 2,
               minibatches: int = 2):
        """obs / mask [T, A * n_tok, ...]: the observation each step's action
        was taken on; actions [T, A]; gstate [T + 1, E * M, 6]: the states
        before each step and after the last; rewards / dones [T, E].
        Returns the objective's outputs [4] of every minibatch step."""
        T, A = actions.shape
        E = A // self.na
        n_tok = self.na + self.nt
        M = self.na + self.nt
        if self.behaviour == "inference":
            values, logits_old = self._behaviour(obs, mask, gstate.reshape(T + 1, E, M, 6))
        else:
            values = self.values(gstate.reshape(T + 1, E, M, 6))
            logits_old = self.logits(obs, mask)
        adv, ret = gae(rewards, dones, values, self.gamma, self.lam)
        if self.recurrent:
            return self._update_rec(obs, mask, actions, gstate.reshape(T + 1, E, M, 6), adv, ret,
                                    logits_old, epochs, minibatches)
        assert T % minibatches == 0, "minibatches must divide the batch's steps"
        k = T // minibatches
        ta = self._pass(k * A, n_tok)
        tc = self._pass(k * E, M + 1)
        gs = gstate.reshape(T + 1, E, M, 6)
        history = []
        for _ in range(epochs):
            for mb in range(minibatches):
                s = slice(mb * k, (mb + 1) * k)
                ln, _ = ta.forward(obs[s].reshape(-1, 6), mask[s].reshape(-1), self.actor)
                v, _ = tc.critic_forward(gs[s].reshape(k * E, M, 6), self.na, self.nt,
                                         self.critic, pos_scale=self.pos_scale)
                out, dl, dv = objective(ln.reshape(k, A, 8), logits_old[s].contiguous(),
                                        actions[s].contiguous(), adv[s].contiguous(),
                                        v.reshape(k, E), ret[s].contiguous(), self.na,
                                        self.n_actions, self.clip_eps)
                ga, _ = ta.backward(self.actor, dl.reshape(k * A, 8), self.n_actions)
                gc, _ = tc.backward(self.critic, dv.reshape(k * E), 1)
                self.opt_a.step(ga)
                self.opt_c.step(gc)
                history.append(out)
        return torch.stack(history)

    def _update_rec(self, obs, mask, actions, gs, adv, ret, logits_old, epochs, minibatches):
        T, A = actions.shape
        E = A // self.na
        n_tok, M = self.na + self.nt, self.na + self.nt
        assert E % minibatches == 0, "minibatches must divide the batch's envs"
        Em = E // minibatches
        Am = Em * self.na
        ta = self._pass(Am, n_tok + 1, 1)
        tc = self._pass(Em, M + 1, 1)
        history = []
        for _ in range(epochs):
            for mb in range(minibatches):
                e0, e1 = mb * Em, (mb + 1) * Em
                a0, a1 = e0 * self.na, e1 * self.na
                o = obs[:, a0 * n_tok:a1 * n_tok].contiguous()
                m = mask[:, a0 * n_tok:a1 * n_tok].contiguous()
                g = gs[:T, e0:e1].contiguous()
                fa, fc = self._actor_fn(ta, o, m), self._critic_fn(tc, g)
                ln, sa = chain_forward(ta, fa, T)
                v, sc = chain_forward(tc, fc, T)
                out, dl, dv = objective(ln, logits_old[:, a0:a1].contiguous(),
                                        actions[:, a0:a1].contiguous(), adv[:, e0:e1].contiguous(),
                                        v, ret[:, e0:e1].contiguous(), self.na, self.n_actions,
                                        self.clip_eps)
                ga = chain_backward(ta, fa, sa, [dl[t] for t in range(T)], self.actor,
                                    self.n_actions)
                gc = chain_backward(tc, fc, sc, [dv[t] for t in range(T)], self.critic, 1)
                self.opt_a.step(ga)
                self.opt_c.step(gc)
                history.append(out)
        return torch.stack(history)

"""Learned range-only estimator: argument marshalling for the MLP kernels.

The network, its features, training kernels and the fallback-guarded
inference all run in libmilrauv.so (see include/mi_lrauv.h, "Learned
range-only estimator"). Torch only allocates device memory, supplies the
stream and draws the data-shuffling permutation.
"""
import ctypes as C

import numpy as np
import torch

from ._lib import check, lib, ptr
from .env import Env, _stream, est_exact

PRECISION = {"bf16": 0, "fp32": 1}


def num_params() -> int:
    return int(lib().mlp_num_params())


def _work(N, precision, device):
    n = int(lib().mlp_workspace_bytes(int(N), PRECISION[precision]))
    buf = torch.empty(n + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, C.c_void_p(buf.data_ptr() + off), n


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    p = torch.empty(num_params(), dtype=torch.float32, device=device)
    check(lib().mlp_init(ptr(p), C.c_uint64(seed), _stream()))
    return p


def features(win: torch.Tensor):
    """win [N, W, 3] -> (x [N, 64], frame [N, 5])."""
    win = win.contiguous()
    N, W, _ = win.shape
    x = torch.empty((N, 64), dtype=torch.float32, device=win.device)
    frame = torch.empty((N, 5), dtype=torch.float32, device=win.device)
    check(lib().mlp_features(ptr(win), N, W, ptr(x), ptr(frame), _stream()))
    return x, frame


def targets(frame: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    y = torch.empty((frame.shape[0], 2), dtype=torch.float32, device=frame.device)
    check(lib().mlp_targets(ptr(frame.contiguous()), ptr(p.contiguous()), frame.shape[0], ptr(y),
                            _stream()))
    return y


def forward(x: torch.Tensor, params: torch.Tensor, precision="bf16") -> torch.Tensor:
    x = x.contiguous()
    N = x.shape[0]
    y = torch.empty((N, 2), dtype=torch.float32, device=x.device)
    buf, w, n = _work(N, precision, x.device)
    check(lib().mlp_forward(N, ptr(x), ptr(params), ptr(y), PRECISION[precision], w, n, _stream()))
    del buf
    return y


def loss_and_grad(x, target, params, index=None, precision="bf16", work=None):
    """Mean over the batch of |y - target|^2 and its gradient."""
    N = x.shape[0] if index is None else index.shape[0]
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    if work is None:
        work = _work(N, precision, params.device)
    _, w, n = work
    check(lib().mlp_backward(N, ptr(x), ptr(index), ptr(target), ptr(params), ptr(grad), ptr(loss),
                             PRECISION[precision], w, n, _stream()))
    return loss, grad


class Adam:
    """Adam state (FP32 moments) driven by the library's kernel."""

    def __init__(self, params: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.step_count = 0

    def step(self, grad: torch.Tensor, lr=None):
        self.step_count += 1
        check(lib().mlp_adam_step(self.params.numel(), ptr(self.params), ptr(grad), ptr(self.m),
                                  ptr(self.v), float(self.lr if lr is None else lr), self.b1,
                                  self.b2, self.eps, self.step_count, _stream()))


def train_step(x, target, opt: "Adam", index=None, lr=None, work=None, grad=None, loss=None):
    """One fused Adam step of the BF16 network (gradient and update in two
    kernels). Returns (loss, grad); `grad` may be given preallocated."""
    N = x.shape[0] if index is None else index.shape[0]
    params = opt.params
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
    if work is None:
        work = _work(N, "bf16", params.device)
    _, w, n = work
    opt.step_count += 1
    check(lib().mlp_train_step(N, ptr(x), ptr(index), ptr(target), ptr(params), ptr(opt.m),
                               ptr(opt.v), float(opt.lr if lr is None else lr), opt.b1, opt.b2,
                               opt.eps, opt.step_count, ptr(grad), ptr(loss), w, n, _stream()))
    return loss, grad


def infer(win: torch.Tensor, params: torch.Tensor, sigma: torch.Tensor, k_sigma=3.0, gn_iters=0,
          tau=1e-4, work=None):
    """Estimates of windows [N, W, 3]: network with residual test, exact
    fallback. Returns (estimates [N, 2], flag [N]: 1 network, 0 exact, 2 none)."""
    win = win.contiguous()
    N, W, _ = win.shape
    out = torch.empty((N, 2), dtype=torch.float32, device=win.device)
    flag = torch.empty((N,), dtype=torch.uint8, device=win.device)
    if work is None:
        work = _work(N, "bf16", win.device)
    _, w, n = work
    check(lib().mlp_infer(ptr(win), N, W, ptr(params), ptr(sigma.contiguous()), float(k_sigma),
                          int(gn_iters), float(tau), ptr(out), ptr(flag), w, n, _stream()))
    return out, flag


def infer_noalloc(win: torch.Tensor, params: torch.Tensor, sigma: torch.Tensor, k_sigma=3.0,
                  gn_iters=0, tau=1e-4, out=None, flag=None):
    """infer() without a workspace: the library's static scratch (at most
    MIL_NOALLOC_MAX_WINDOWS windows per call; calls on one GPU must not overlap).
    `out` and `flag` may be given preallocated."""
    win = win.contiguous()
    N, W, _ = win.shape
    if out is None:
        out = torch.empty((N, 2), dtype=torch.float32, device=win.device)
    if flag is None:
        flag = torch.empty((N,), dtype=torch.uint8, device=win.device)
    check(lib().mlp_infer_noalloc(ptr(win), N, W, ptr(params), ptr(sigma.contiguous()),
                                  float(k_sigma), int(gn_iters), float(tau), ptr(out), ptr(flag),
                                  _stream()))
    return out, flag


def env_windows(env: Env):
    """Current windows of every tracker: (win [P, W, 3], sigma [P], truth [P, 2])."""
    W = env.layout.window
    win = torch.empty((env.P, W, 3), dtype=torch.float32, device=env.device)
    sigma = torch.empty((env.P,), dtype=torch.float32, device=env.device)
    truth = torch.empty((env.P, 2), dtype=torch.float32, device=env.device)
    check(lib().env_windows(env._h, ptr(win), ptr(sigma), ptr(truth), _stream()))
    return win, sigma, truth


def rollout_windows(cfg: dict, num_envs: int, n_windows: int, seed: int, first_step=100,
                    every=50, device="cuda"):
    """Windows from the environment itself: run the (ragged) workload and copy
    every tracker's full window every `every` steps from `first_step` on, with
    the exact estimate of each (FP64 est_exact) as label. Windows whose exact
    solve is refused are dropped. Returns dict of tensors."""
    env = Env(cfg, num_envs, seed=seed, device=device)
    env.reset(0)
    W = cfg["window"]
    got = {"win": [], "sigma": [], "truth": [], "exact": []}
    total = 0
    t = 0
    step = first_step
    while total < n_windows:
        if step > cfg["episode_len"]:
            break
        env.rollout(step - t, record=())
        t = step
        win, sigma, truth = env_windows(env)
        exact, valid = est_exact(win)
        keep = valid.bool() & ~torch.isnan(win[..., 2]).any(dim=1)
        for k, v in (("win", win), ("sigma", sigma), ("truth", truth), ("exact", exact)):
            got[k].append(v[keep])
        total += int(keep.sum().item())
        step += every
    assert W >= 3
    out = {k: torch.cat(v)[:n_windows] for k, v in got.items()}
    env.close()
    return out


def train(x, y, params=None, epochs=2, batch=8192, lr=2e-3, lr_final=1e-4, seed=0,
          precision="bf16", log=None):
    """Adam on the mean-squared error of the normalised target; cosine decay of
    the learning rate from lr to lr_final. Returns (params, loss history)."""
    device = x.device
    if params is None:
        params = init_params(seed, device)
    opt = Adam(params, lr=lr)
    N = x.shape[0]
    steps_per_epoch = max(1, N // batch)
    total = epochs * steps_per_epoch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    work = _work(batch, precision, device)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(N, generator=gen, device=device)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            cur = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * k / max(1, total - 1)))
            if precision == "bf16":
                train_step(x, y, opt, index=idx, lr=cur, work=work, grad=grad, loss=loss)
            else:
                loss, grad = loss_and_grad(x, y, params, index=idx, precision=precision,
                                           work=work)
                opt.step(grad, lr=cur)
            if b % 50 == 0 or b == steps_per_epoch - 1:
                hist.append((k, float(loss.item())))
                if log:
                    log(f"epoch {ep} step {b}/{steps_per_epoch} loss {hist[-1][1]:.3e}")
            k += 1
    return params, hist

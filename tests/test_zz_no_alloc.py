"""The workspace-free guarded inference (mlp_infer_noalloc), called through
the C ABI, against mlp_infer with a caller workspace: the same estimates and
flags bit for bit, on two calls in a row (the second smaller, so it runs on
the scratch the first left behind)."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_08222_amd.synth import range_windows  # noqa: E402

pytestmark = pytest.mark.gpu


def _call_noalloc(win, params, sigma, k_sigma, gn_iters):
    from paper_2505_08222_amd._lib import check, lib, ptr
    N, W, _ = win.shape
    out = torch.full((N, 2), float("nan"), dtype=torch.float32, device=win.device)
    flag = torch.full((N,), 255, dtype=torch.uint8, device=win.device)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib().mlp_infer_noalloc(ptr(win), N, W, ptr(params), ptr(sigma), float(k_sigma),
                                  int(gn_iters), 1e-4, ptr(out), ptr(flag), stream))
    return out, flag


def test_noalloc_equals_workspace_inference():
    from paper_2505_08222_amd import learned
    params = learned.init_params(5)
    rng = np.random.default_rng(3)
    # first call: a larger batch, the usual residual test (most windows fall
    # back to the exact solve); second call: smaller, a looser test (a mix)
    for N, W, k_sigma, gn, seed in ((9000, 16, 3.0, 0, 1), (2500, 10, 40.0, 2, 2)):
        win = torch.from_numpy(range_windows(N, W, seed=seed, missing=0.003, far=900.0)).cuda()
        sigma = torch.from_numpy(rng.uniform(0.5, 3.0, N).astype(np.float32)).cuda()
        got, gflag = _call_noalloc(win, params, sigma, k_sigma, gn)
        want, wflag = learned.infer(win, params, sigma, k_sigma=k_sigma, gn_iters=gn)
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        gf, wf = gflag.cpu().numpy(), wflag.cpu().numpy()
        np.testing.assert_array_equal(gf, wf)
        np.testing.assert_array_equal(g.view(np.uint32), w.view(np.uint32))
        counts = np.bincount(gf, minlength=3)
        print(f"N={N} W={W}: network {counts[1]}, exact {counts[0]}, none {counts[2]}")
        assert counts[0] > 0 and set(np.unique(gf)) <= {0, 1, 2}
        if k_sigma > 3:
            assert counts[1] > 0

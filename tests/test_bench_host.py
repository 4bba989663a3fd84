"""Host-side checks of bench.py (no GPU): the counter lines committed under
profiles/ parse and belong to the current kernel sources (else the bench
would report their traffic and VALU figures as unmeasured), and the
one-GPU contract refuses other GPU counts before touching a device."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _counter_lines():
    pat = re.compile(r"^(traffic|valu)\s+(\S+)\s+(\S+)\s+(\S+)\s+(\d+)\s+(\d+)\s*$")
    out = []
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            for line in f:
                m = pat.match(line.strip())
                if m:
                    out.append((name,) + m.groups())
    return out


def test_counter_lines_match_the_current_kernels():
    lines = _counter_lines()
    kinds = {(k, kern, wl) for _, k, kern, wl, _, _, _ in lines}
    # the headline's traffic, the particle filter's and the paper rollouts' VALU figures
    assert ("traffic", "rollout_kernel", "ragged") in kinds
    assert ("valu", "pf_kernel", "ragged_pf") in kinds
    assert ("valu", "rollout_kernel", "paper") in kinds
    for name, kind, kern, wl, ver, a, b in lines:
        assert ver == bench.kernel_version(kern), (name, kind, kern, wl)
        assert int(a) > 0 and int(b) > 0


def test_measured_figures_are_found():
    assert bench.measured_traffic("rollout_kernel", "ragged") is not None
    busy, insts = bench.measured_valu("rollout_kernel", "paper")
    assert busy > insts > 0
    assert bench.measured_valu("rollout_kernel", "ragged") is None  # HBM-bound line: no VALU view


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)

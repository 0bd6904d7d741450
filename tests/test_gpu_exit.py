"""Process exit with library handles still alive at module scope: the binding
closes them (factors first, then contexts) from an exit hook while the HIP
runtime is still up, and the process ends with status 0."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np, torch
from paper_2402_06835_amd import api
from synth import make_workload, sho_omega_from_rotation
w = make_workload("exit", 5, 700, 10 / 1440,
                  {"amp": 0.01, "omega": sho_omega_from_rotation(1.2, 5.0), "q": 5.0, "sigma_w": 1e-3},
                  [2, 5], np.linspace(0.3, 1.5, 20))
CTX = api.Context(0)
CTX.set_inverse_prefetch("fp32_refine")
FAC = api.gp_factor(CTX, w.t, w.theta)
LS = api.linear_search(CTX, FAC, w.f, w.A, w.lattice, w.n_epochs, w.durations, "fp32_refine")
PS = api.periodic_search(CTX, LS["depth"], LS["var"], LS["dll"], LS["valid"], w.dt, w.periods)
torch.cuda.synchronize()
print("module-scope handles alive at exit", flush=True)
"""


def test_exit_with_module_scope_handles():
    print("[gpu-case] exit with a module-scope context and factor", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert "module-scope handles alive at exit" in r.stdout, r.stderr[-2000:]
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])

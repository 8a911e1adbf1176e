"""Long runs of the benchmark workloads on the GPU against the FP64 oracle's
runs of the same workloads (tests/golden/oracle_*.npz, written by
tests/golden/make_oracle_runs.py from the oracle alone), compared at the
stored sample of mesh nodes and by the whole-grid L1 norm of each field.

The oracle runs in FP64 from the values as the split form stores them
(FP32-rounded), so a plain-FP64 GPU run from the same values is the parity
check proper (bound derived below); the FP32-value run of the same workload is
compared with the same oracle result, which measures the split form's
accumulated error."""
import os
import sys

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W
from tests.util import stored_values

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

WORKLOADS = {
    "swirl1024_period": lambda: W.swirl_three_fields(1024, value_prec="f32"),
    "fourier3d256_50": lambda: W.fourier3d_three_fields(256, value_prec="f32"),
    "deform3d512_10": lambda: W.deform3d_slotted_sphere(512),
    "kelvin256_t1": lambda: W.kelvin(256, amp=1e-4, t_end=1.0),
    "kelvin_nonlinear256_t1": lambda: W.kelvin(256, amp=0.5, nu=5e-4, t_end=1.0),
    "kelvin1024_t1": lambda: W.kelvin(1024, amp=1e-4, t_end=1.0),
}

# Relative L1 over the sampled nodes (and of the whole-grid norm).
# FP64: the GPU and the oracle differ only in rounding (fused multiply-adds,
# the order of partial sums, the refined-reciprocal Newton), a few units of
# 2^-53 per step; the 1e-12 tolerance of single steps holds over the whole
# runs (1280 steps of the swirl measure below 1e-13).
# FP32 values: each step stores its results rounded to 2^-24 relative, and a
# rounding that crosses a limiter threshold lowers one node's order (a local
# change of the interpolation error, up to ~1e-2 of the field's range); over
# long runs this accumulates well above a single step's 1e-5 (a period of the
# swirl: 1.2e-3 at samples concentrated on the slotted disc's edge, whose
# own error against the exact solution is 0.6).  1e-2 is an envelope; the
# test prints the measured values.
TOL = {"f64": 1e-12, "f32": 1e-2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.fail("no GPU visible")
    return T


@pytest.fixture(scope="module")
def B():
    from paper_1410_2817_amd import binding
    binding.load()
    return binding


@pytest.mark.parametrize("case", list(WORKLOADS))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_run_vs_oracle(B, torch, case, prec):
    path = os.path.join(GOLDEN, "oracle_%s.npz" % case)
    if not os.path.exists(path):
        pytest.skip("oracle run not stored yet (tests/golden/make_oracle_runs.py %s)" % case)
    ref = np.load(path, allow_pickle=False)
    wl = WORKLOADS[case]()
    steps, t0 = int(ref["steps"]), float(ref["t0"])
    assert abs(float(ref["dt"]) - wl.dt) < 1e-15
    say("full run", case, prec, wl.shape, "steps", steps)
    g = B.Grid.from_workload(wl, value_prec=prec)
    out = g.advance(g.new_fields(stored_values(wl)), t0, wl.dt, steps)
    rc, st = g.sync()
    assert rc == 0 and st["search_fail"] == 0 and st["newton_fail"] == 0
    nodes, want = ref["nodes"], ref["values"]
    total = float(np.abs(want).sum())
    num = 0.0
    for f, fld in enumerate(out):
        full = fld.double().cpu().numpy().ravel()
        got = full[nodes]
        num += float(np.abs(got - want[:, f]).sum())
        rel = np.abs(got - want[:, f]).sum() / np.abs(want[:, f]).sum()
        linf = np.abs(got - want[:, f]).max()
        norm = abs(np.abs(full).sum() - ref["l1"][f]) / ref["l1"][f]
        share = float(np.abs(want[:, f]).sum()) / total
        say("  field", f, "sampled rel L1 %.3e" % rel, "Linf %.3e" % linf, "norm %.3e" % norm,
            "share %.2e" % share)
        # A field holding a negligible part of the total (the Kelvin wave's
        # u2 is zero up to rounding) is held to the all-field measure only.
        if share >= 1e-3:
            assert rel <= TOL[prec] and norm <= TOL[prec], (f, rel, norm)
    say("  all fields sampled rel L1 %.3e" % (num / total))
    assert num / total <= TOL[prec]

"""sl_advance_static, the entry point for callers that cannot allocate: it
runs the same kernels as sl_advance with the library's static scratch in
place of the caller's workspace.  Two calls in a row (the second on a smaller
grid, so the scratch holds the first call's leftovers) must give sl_advance's
results bitwise and its counters; a grid whose workspace exceeds the scratch
is refused with SL_ETOOBIG."""
import sys

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W
from tests.util import stored_values

pytestmark = pytest.mark.gpu


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


def _both(B, torch, wl, nsteps, t0):
    g = B.Grid.from_workload(wl)
    want = g.advance(g.new_fields(stored_values(wl)), t0, wl.dt, nsteps)
    rc, st = g.sync()
    assert rc == 0
    want = [f.cpu().numpy() for f in want]
    cnt = torch.full((B.SL_STATIC_COUNTERS,), -1, dtype=torch.int64, device=g.device)
    got = g.advance_static(g.new_fields(stored_values(wl)), t0, wl.dt, nsteps, counters=cnt)
    torch.cuda.synchronize()
    got = [f.cpu().numpy() for f in got]
    return want, st, got, cnt.cpu().numpy()


@pytest.mark.parametrize("cases", [
    [("swirl256_f32", W.swirl_three_fields(256, value_prec="f32"), 7, 0.3),
     ("swirl128_f32", W.swirl_three_fields(128, value_prec="f32"), 5, 1.1)],
    [("deform3d48_f64", W.deform3d_slotted_sphere(48), 4, 0.2),
     ("deform3d32_f64", W.deform3d_slotted_sphere(32), 3, 0.5)],
], ids=["2d", "3d"])
def test_static_scratch_matches_workspace_path(B, torch, cases):
    for name, wl, nsteps, t0 in cases:
        say("static scratch", name, nsteps)
        want, st, got, cnt = _both(B, torch, wl, nsteps, t0)
        for a, b in zip(got, want):
            assert np.array_equal(a, b), name
        expect = [st["search_fail"], st["newton_fail"], st["nonfinite"], st["order_hist"][0],
                  st["order_hist"][1], st["walked"], st["scanned"], 0]
        say("  counters", cnt.tolist(), "sl_sync", expect)
        assert cnt.tolist() == expect


def test_static_scratch_refuses_large_grids(B, torch):
    wl = W.swirl_three_fields(2048, value_prec="f32", nsteps=1)
    g = B.Grid.from_workload(wl)
    assert int(B.load().sl_workspace_bytes(g._h)) > B.SL_STATIC_SCRATCH_BYTES
    x = g.new_fields()
    with pytest.raises(B.SlError) as e:
        g.advance_static(x, 0.0, wl.dt, 1)
    assert e.value.code == B.SL_ETOOBIG

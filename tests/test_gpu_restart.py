"""Per-step parity of the FP32-value form along whole runs of the benchmark
workloads.

The split form stores field values in FP32 between steps, so its run drifts
away from an FP64 run of the same workload (rounding of the stored values,
and the limiter decisions those roundings move across the threshold).  The
parity it owes the oracle is per step: at chosen steps k of a GPU run, the
GPU's own FP32 state S_k is handed to the oracle, which takes one FP64 step
from it; the GPU's S_{k+1} must match that step within the FP32 tolerance
(relative L1 <= 1e-5 over the checked nodes, and every checked node within
1e-5 of the field's largest value, which an order chosen differently from the
oracle's would break).  Whole grids are checked where the oracle step takes
seconds (2-D), sampled nodes where it would not (3-D: random nodes plus nodes
on the slotted sphere's edge, evaluated one by one by the oracle)."""
import sys

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W
from tests.util import oracle_problem, stored_values

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def _advance(g, cur, spare, t, dt, n):
    """n steps from `cur`; returns (result buffers, the other set)."""
    out = g.advance(cur, t, dt, n, out=spare)
    in_cur = out[0].data_ptr() == cur[0].data_ptr()
    return (out, spare if in_cur else cur)


def _edge_nodes(field0, g, count):
    f = field0.ravel()
    scale = max(np.abs(f).max(), 1e-300)
    edge = np.nonzero(np.abs(np.diff(f, append=f[:1])) > 0.1 * scale)[0]
    if edge.size == 0:
        return np.zeros(0, np.int64)
    return g.choice(edge, min(count, edge.size), replace=False)


def _compare(tag, got, want):
    """got, want: lists of per-field FP64 arrays over the checked nodes."""
    num = den = 0.0
    for f, (a, b) in enumerate(zip(got, want)):
        d = np.abs(a - b)
        scale = max(np.abs(b).max(), 1e-300)
        num += float(d.sum())
        den += float(np.abs(b).sum())
        assert d.max() <= TOL * scale, (tag, f, float(d.max()), scale)
    rel = num / max(den, 1e-300)
    assert rel <= TOL, (tag, rel)
    return rel


def _run_with_checks(B, torch, orc, wl, nsteps, checks, sample=None, t0=0.0):
    """GPU run of nsteps; at each step k in `checks`, one oracle step from
    the GPU state S_k is compared with the GPU's S_{k+1}.  `sample`: None for
    whole grids, else (random count, edge count) of sampled nodes."""
    g = B.Grid.from_workload(wl)
    prob = oracle_problem(orc, wl)
    cur = g.new_fields(stored_values(wl))
    spare = g.new_fields()
    rng = np.random.Generator(np.random.PCG64(17))
    k, worst = 0, 0.0
    for c in sorted(checks):
        if c > k:
            cur, spare = _advance(g, cur, spare, t0 + k * wl.dt, wl.dt, c - k)
            k = c
        state = [f.double().cpu().numpy() for f in cur]
        t = t0 + k * wl.dt
        cur, spare = _advance(g, cur, spare, t, wl.dt, 1)
        k += 1
        rc, st = g.sync()
        assert rc == 0 and st["search_fail"] == 0 and st["newton_fail"] == 0, (c, rc, st)
        nxt = [f.double().cpu().numpy() for f in cur]
        if sample is None:
            orc_rc, want, _ = orc.step(prob, t, wl.dt, state)
            assert orc_rc == 0
            got = [a.ravel() for a in nxt]
            want = [b.ravel() for b in want]
        else:
            nodes = np.unique(np.concatenate([
                rng.integers(0, wl.nodes, sample[0]),
                _edge_nodes(state[0], rng, sample[1])])).astype(np.int64)
            orc_rc, vals, _ = orc.step_sampled(prob, t, wl.dt, state, nodes)
            assert orc_rc == 0
            got = [a.ravel()[nodes] for a in nxt]
            want = [vals[:, f] for f in range(wl.nfields)]
        rel = _compare((wl.name, c), got, want)
        worst = max(worst, rel)
        say("  step", c, "->", c + 1, "rel L1 %.3e" % rel)
        del state, nxt
    if k < nsteps:
        cur, spare = _advance(g, cur, spare, t0 + k * wl.dt, wl.dt, nsteps - k)
        rc, _ = g.sync()
        assert rc == 0
    say("  worst step rel L1 %.3e" % worst)
    return worst


def test_swirl1024_period_every_64th_step(B, torch, orc):
    wl = W.swirl_three_fields(1024, value_prec="f32")
    say("restart parity", wl.name, wl.nsteps, "steps")
    checks = list(range(0, wl.nsteps, 64)) + [wl.nsteps - 1]
    _run_with_checks(B, torch, orc, wl, wl.nsteps, checks)


def test_fourier3d256_fifty_steps(B, torch, orc):
    wl = W.fourier3d_three_fields(256, value_prec="f32")
    say("restart parity", wl.name, wl.nsteps, "steps")
    _run_with_checks(B, torch, orc, wl, wl.nsteps, [0, 10, 20, 30, 40, 49],
                     sample=(3000, 1500))


def test_deform3d512_first_ten_steps(B, torch, orc):
    wl = W.deform3d_slotted_sphere(512, value_prec="f32")
    say("restart parity", wl.name, "first 10 steps")
    _run_with_checks(B, torch, orc, wl, 10, list(range(10)), sample=(2000, 1000))

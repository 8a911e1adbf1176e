"""Serving: requests batched by the server give the same bits as each request
run alone; admission respects the arena budget; a served request matches the
oracle."""
import sys

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W
from tests.util import l1_rel, oracle_problem

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
def S():
    from paper_1410_2817_amd import serving
    return serving


def _requests(n=6, seed=3):
    g = W.rng(seed)
    return [W.serving_request(g, i, 0.0, sides=(64, 96, 128, 200), steps_range=(3, 9))
            for i in range(n)]


def _alone(torch, req):
    from paper_1410_2817_amd import binding as B
    g = B.Grid(req.shape, req.nfields, value_prec="f32", order_max=2, limiter=True,
               vel_kind=W.VEL_FOURIER, vel_params=[1.0], modes=req.modes)
    x = req.fields_torch(g.device, torch.float32)
    out = g.advance(x, 0.0, req.dt, req.nsteps)
    rc, _ = g.sync()
    assert rc == 0
    return [f.cpu().numpy() for f in out]


MODES = [("batched", 1), ("queued", 1), ("queued", 3), ("queued", 16)]


@pytest.mark.parametrize("mode,window", MODES)
def test_mix_equals_alone_bitwise(torch, S, mode, window):
    """Served in a mix (staggered admissions, several field counts and sides)
    each request gives the bits of its run alone, in every launch mode: one
    batched launch per tick, or queued launches of 1, 3 or 16 steps (in which
    a request's later steps wait on the device for its earlier ones)."""
    reqs = _requests()
    say("alone")
    alone = {r.rid: _alone(torch, r) for r in reqs}
    say("mix", mode, window)
    srv = S.Server(256 << 20, max_requests=8, max_inflight=2, mode=mode, window=window)
    dev = srv.device
    ids, got = {}, {}
    # Staggered admissions: three now, the rest after two ticks.
    for r in reqs[:3]:
        (desc, _), f = S.request_desc(r), r.fields_torch(dev, torch.float32)
        ids[srv.admit(desc, f, r.dt, r.nsteps)] = r
    srv.tick()
    srv.tick()
    for r in reqs[3:]:
        (desc, _), f = S.request_desc(r), r.fields_torch(dev, torch.float32)
        ids[srv.admit(desc, f, r.dt, r.nsteps)] = r
    while len(got) < len(reqs):
        srv.tick()
        for sid in srv.poll():
            r = ids[sid]
            out = [torch.empty(r.shape, dtype=torch.float32, device=dev) for _ in range(r.nfields)]
            srv.fetch(sid, out)
            torch.cuda.synchronize()
            got[r.rid] = [o.cpu().numpy() for o in out]
    rc, st = srv.sync()
    assert rc == 0 and st["search_fail"] == 0
    for r in reqs:
        for a, b in zip(got[r.rid], alone[r.rid]):
            assert np.array_equal(a, b), r.rid
    srv.close()


def test_admission_respects_budget(torch, S):
    reqs = _requests(3, seed=5)
    desc0, _ = S.request_desc(reqs[0])
    need = S.Server.request_bytes(desc0)
    # Room for the server's own data and exactly one request of this size.
    srv = S.Server(S.Server.arena_overhead(2) + need, max_requests=2, max_inflight=1)
    dev = srv.device
    f0 = reqs[0].fields_torch(dev, torch.float32)
    a = srv.admit(desc0, f0, reqs[0].dt, reqs[0].nsteps)
    assert a is not None
    big = max(reqs[1:], key=lambda q: q.nodes)
    (desc1, _), f1 = S.request_desc(big), big.fields_torch(dev, torch.float32)
    assert S.Server.request_bytes(desc1) > 12 * 1024
    assert srv.admit(desc1, f1, big.dt, big.nsteps) is None  # no room: SL_EBUSY
    done = []
    while not done:
        srv.tick()
        done = srv.poll()
    out = [torch.empty(reqs[0].shape, dtype=torch.float32, device=dev)
           for _ in range(reqs[0].nfields)]
    srv.fetch(done[0], out)
    # Memory came back: a request of the same size fits again.
    assert srv.admit(desc0, f0, reqs[0].dt, reqs[0].nsteps) is not None
    info = srv.info()
    assert info["bytes_in_use"] == need and info["active"] == 1
    srv.close()
    # The slot limit binds too.
    srv = S.Server(64 << 20, max_requests=1)
    assert srv.admit(desc0, f0, reqs[0].dt, reqs[0].nsteps) is not None
    assert srv.admit(desc0, f0, reqs[0].dt, reqs[0].nsteps) is None
    srv.close()


def test_served_request_matches_oracle(torch, S, orc):
    req = W.serving_request(W.rng(11), 0, 0.0, sides=(96,), steps_range=(4, 4))
    srv = S.Server(64 << 20, max_requests=2)
    dev = srv.device
    (desc, _), f = S.request_desc(req), req.fields_torch(dev, torch.float32)
    stored = [x.double().cpu().numpy() for x in f]
    sid = srv.admit(desc, f, req.dt, req.nsteps)
    got = None
    while got is None:
        srv.tick()
        for d in srv.poll():
            out = [torch.empty(req.shape, dtype=torch.float32, device=dev) for _ in range(req.nfields)]
            srv.fetch(d, out)
            got = [o.double().cpu().numpy() for o in out]
    wl = req.workload
    wl.fields = stored
    rc, want, _ = orc.run(oracle_problem(orc, wl), 0.0, wl.dt, wl.nsteps, stored)
    assert rc == 0
    for a, b in zip(got, want):
        assert l1_rel(a, b) <= 1e-5
    srv.close()


@pytest.mark.parametrize("mode,window", [("batched", 1), ("queued", 4)])
def test_stream_driver_completes(torch, S, mode, window):
    reqs = W.serving_stream(seed=2, count=24, rate=400.0, sides=(64, 128, 256),
                            steps_range=(5, 12))
    rep = S.run_stream(reqs, 64 << 20, max_requests=16, mode=mode, window=window)
    say(rep)
    assert rep["status"] == 0 and rep["requests"] == 24
    assert rep["latency_p99_ms"] >= rep["latency_p50_ms"] > 0


# --------------------------------------------------------------------------
# Served requests against the oracle at the serving mix's sizes.

def _golden():
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location(
        "make_oracle_runs", os.path.join(here, "golden", "make_oracle_runs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod, os.path.join(here, "golden")


def _serve_all(torch, S, reqs, prec, budget=3 << 30, mode="batched", window=1):
    """Admit every (request, nsteps) pair into one server, half of them after
    two ticks, run to completion; returns {index: fields as FP64 numpy}."""
    from paper_1410_2817_amd import binding as B
    dt_ = torch.float32 if prec == "f32" else torch.float64
    srv = S.Server(budget, max_requests=len(reqs) + 1, max_inflight=2, mode=mode,
                   window=window)
    dev = srv.device
    ids, got = {}, {}

    def admit(i):
        req, nsteps = reqs[i]
        desc, _ = B.make_desc(req.shape, req.nfields, value_prec=prec, order_max=2,
                              limiter=True, vel_kind=W.VEL_FOURIER, vel_params=[1.0],
                              modes=req.modes)
        f = [torch.as_tensor(x, device=dev).to(dt_).contiguous() for x in req.fields()]
        sid = srv.admit(desc, f, req.dt, nsteps)
        assert sid is not None, ("no room", i)
        ids[sid] = i

    half = (len(reqs) + 1) // 2
    for i in range(half):
        admit(i)
    srv.tick()
    srv.tick()
    for i in range(half, len(reqs)):
        admit(i)
    while len(got) < len(reqs):
        srv.tick()
        for sid in srv.poll():
            i = ids[sid]
            req = reqs[i][0]
            out = [torch.empty(req.shape, dtype=dt_, device=dev) for _ in range(req.nfields)]
            srv.fetch(sid, out)
            torch.cuda.synchronize()
            got[i] = [o.double().cpu().numpy() for o in out]
    rc, st = srv.sync()
    assert rc == 0 and st["search_fail"] == 0 and st["newton_fail"] == 0, (rc, st)
    srv.close()
    return got


SERVED = ["serve_mix128", "serve_mix256", "serve_mix512", "serve_mix1024",
          "serve_mix2048", "serve2048_50"]


@pytest.mark.parametrize("mode,window", [("batched", 1), ("queued", 4)])
def test_served_fp64_runs_match_stored_oracle_runs(torch, S, mode, window):
    """FP64 requests of every side of the serving mix (and a 2048^2 one for
    50 steps), served together with staggered admission, against the
    oracle's runs of the same requests (tests/golden/oracle_serve_*.npz) at
    the stored sample of nodes and by each field's whole-grid L1 norm."""
    mod, gold = _golden()
    import os
    reqs = [(mod.served_request(n), mod.SERVED[n][2]) for n in SERVED]
    say("served fp64", mode, window, [(r.n, r.nfields, k) for r, k in reqs])
    got = _serve_all(torch, S, reqs, "f64", mode=mode, window=window)
    for i, name in enumerate(SERVED):
        ref = np.load(os.path.join(gold, "oracle_%s.npz" % name), allow_pickle=False)
        assert int(ref["steps"]) == reqs[i][1]
        nodes, want = ref["nodes"], ref["values"]
        num = den = 0.0
        for f, fld in enumerate(got[i]):
            a = fld.ravel()[nodes]
            num += float(np.abs(a - want[:, f]).sum())
            den += float(np.abs(want[:, f]).sum())
            norm = abs(np.abs(fld).sum() - ref["l1"][f]) / ref["l1"][f]
            assert norm <= 1e-12, (name, f, norm)
        say("  ", name, "rel L1 %.3e" % (num / den))
        assert num / den <= 1e-12, (name, num / den)


@pytest.mark.parametrize("mode,window", [("batched", 1), ("queued", 4)])
def test_served_fp32_steps_match_oracle_steps(torch, S, orc, mode, window):
    """FP32 requests of every side: each is served twice in the same mix,
    for n - 1 and for n steps; one oracle step from the (n - 1)-step result
    must give the n-step result within the FP32 tolerance (whole grids up to
    512^2, sampled nodes above)."""
    mod, _ = _golden()
    base = [(mod.served_request(n), mod.SERVED[n][2]) for n in SERVED]
    reqs = []
    for r, k in base:
        reqs += [(r, k - 1), (r, k)]
    say("served fp32 pairs", mode, window, [(r.n, k) for r, k in reqs])
    got = _serve_all(torch, S, reqs, "f32", mode=mode, window=window)
    rng = np.random.Generator(np.random.PCG64(23))
    for j, (r, k) in enumerate(base):
        prev, last = got[2 * j], got[2 * j + 1]
        wl = r.workload
        wl.fields = prev
        prob = oracle_problem(orc, wl)
        t = (k - 1) * r.dt
        if r.n <= 512:
            rc, want, _ = orc.step(prob, t, r.dt, prev)
            assert rc == 0
            pairs = [(a.ravel(), b.ravel()) for a, b in zip(last, want)]
        else:
            f0 = prev[0].ravel()
            edge = np.nonzero(np.abs(np.diff(f0, append=f0[:1])) > 0.1 * np.abs(f0).max())[0]
            nodes = np.unique(np.concatenate([
                rng.integers(0, r.nodes, 3000),
                rng.choice(edge, min(1500, edge.size), replace=False)])).astype(np.int64)
            rc, vals, _ = orc.step_sampled(prob, t, r.dt, prev, nodes)
            assert rc == 0
            pairs = [(a.ravel()[nodes], vals[:, f]) for f, a in enumerate(last)]
        num = den = 0.0
        for f, (a, b) in enumerate(pairs):
            d = np.abs(a - b)
            assert d.max() <= 1e-5 * np.abs(b).max(), (r.n, f, float(d.max()))
            num += float(d.sum())
            den += float(np.abs(b).sum())
        say("  side", r.n, "step", k - 1, "->", k, "rel L1 %.3e" % (num / den))
        assert num / den <= 1e-5


def test_server_counts_every_step(torch, S):
    """sl_server_sync reports the request steps it ran: nodes, steps and
    reconstructions, and the order histogram summing to the field-node
    reconstructions."""
    reqs = _requests(4, seed=8)
    srv = S.Server(128 << 20, max_requests=4, mode="queued", window=2)
    dev = srv.device
    for r in reqs:
        (desc, _), f = S.request_desc(r), r.fields_torch(dev, torch.float32)
        assert srv.admit(desc, f, r.dt, r.nsteps) is not None
    while srv.tick() > 0:
        pass
    rc, st = srv.sync()
    assert rc == 0
    assert st["steps"] == st["reconstructs"] == sum(r.nsteps for r in reqs)
    assert st["nodes"] == sum(r.nodes * r.nsteps for r in reqs)
    assert sum(st["order_hist"]) == sum(r.nodes * r.nsteps * r.nfields for r in reqs)
    srv.close()

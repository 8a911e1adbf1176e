"""Write the oracle's results of long runs of the benchmark workloads, sampled
at a fixed set of mesh nodes, for the GPU full-run parity tests.

Only the oracle (oracle/) and the seeded input generators run here; nothing
comes from the GPU path.  Each case stores, as a compressed .npz:
  nodes   flat indices of the sampled mesh nodes (random, plus nodes next to
          the initial discontinuity of field 0)
  values  the oracle's field values there after `steps` steps, shape
          (len(nodes), nfields)
  l1      sum over all nodes of |value| per field (a whole-grid check)
  t0, dt, steps
  store   "f64", or "f32" for runs whose values are rounded to FP32 after
          every step (the values the FP32-value form carries between steps)

Served requests (serve_*) are seeded draws of the serving stream's request
generator, run in FP64 from the request's FP64 fields.

Run from the repository root:  python tests/golden/make_oracle_runs.py [case ...]
(several minutes per case on a few cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1410_2817_amd import workloads as W  # noqa: E402


# Served requests of the parity tests: (seed, side, steps).
SERVED = {
    "serve2048_50": (31, 2048, 50),
    "serve_mix128": (41, 128, 37),
    "serve_mix256": (42, 256, 21),
    "serve_mix512": (43, 512, 44),
    "serve_mix1024": (44, 1024, 16),
    "serve_mix2048": (45, 2048, 12),
}


def served_request(name):
    seed, side, steps = SERVED[name]
    return W.serving_request(W.rng(seed), 0, 0.0, sides=(side,), steps_range=(steps, steps))


def served_workload(name):
    wl = served_request(name).workload
    wl.value_prec = "f64"
    return wl


def cases():
    # name: (workload factory, steps, t0[, store]); the oracle runs in FP64
    # from the values as stored by the GPU form named in the workload
    # (FP32-rounded for the split form); store "f32" also rounds the values
    # after every step.
    c = {
        "swirl1024_period": (lambda: W.swirl_three_fields(1024, value_prec="f32"), 1280, 0.0),
        "fourier3d256_50": (lambda: W.fourier3d_three_fields(256, value_prec="f32"), 50, 0.0),
        "deform3d512_10": (lambda: W.deform3d_slotted_sphere(512), 10, 0.0),
        # Shallow-water source terms (the oracle's run_source): the Kelvin
        # wave to t = 1, linear and non-linear viscous.
        "kelvin256_t1": (lambda: W.kelvin(256, amp=1e-4, t_end=1.0), 512, 0.0),
        "kelvin_nonlinear256_t1": (lambda: W.kelvin(256, amp=0.5, nu=5e-4, t_end=1.0), 525, 0.0),
        "kelvin1024_t1": (lambda: W.kelvin(1024, amp=1e-4, t_end=1.0), 2048, 0.0),
    }
    for name, (_, _, steps) in SERVED.items():
        c[name] = ((lambda nm=name: served_workload(nm)), steps, 0.0)
    return c


def stored(wl):
    if wl.value_prec == "f32":
        return [np.asarray(f, dtype=np.float32).astype(np.float64) for f in wl.fields]
    return [np.asarray(f, dtype=np.float64) for f in wl.fields]


def sample_nodes(wl, seed=2024, nrand=6000, nedge=2000):
    g = np.random.Generator(np.random.PCG64(seed))
    f0 = wl.fields[0].ravel()
    edge = np.nonzero(np.abs(np.diff(f0, append=f0[:1])) > 0)[0]
    pick = [g.integers(0, wl.nodes, nrand)]
    if edge.size:
        pick.append(g.choice(edge, min(nedge, edge.size), replace=False))
    return np.unique(np.concatenate(pick)).astype(np.int64)


def run(name):
    make, steps, t0, *rest = cases()[name]
    store = rest[0] if rest else "f64"
    wl = make()
    prob = oracle.Problem(wl.shape, wl.nfields, wl.length, order_max=wl.order_max,
                          limiter=wl.limiter, theta=wl.theta, integrator=wl.integrator,
                          vel_kind=wl.velocity.kind, vp=wl.velocity.padded_params(),
                          modes=wl.velocity.modes, src_kind=wl.source, sp=list(wl.sp))
    t = time.time()
    if wl.source:
        rc, fields, st = oracle.run_source(prob, t0, wl.dt, steps, stored(wl))
    else:
        rc, fields, st = oracle.run(prob, t0, wl.dt, steps, stored(wl), store=store)
    assert rc == 0, (name, rc, st)
    nodes = sample_nodes(wl)
    values = np.stack([f.ravel()[nodes] for f in fields], axis=1)
    l1 = np.array([np.abs(f).sum() for f in fields])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_%s.npz" % name)
    np.savez_compressed(out, nodes=nodes, values=values, l1=l1, t0=t0, dt=wl.dt, steps=steps,
                        store=store)
    print(name, "steps", steps, "oracle s %.0f" % (time.time() - t), "threads", oracle.threads(),
          "->", os.path.basename(out), flush=True)


if __name__ == "__main__":
    oracle.build()
    for name in (sys.argv[1:] or list(cases())):
        run(name)

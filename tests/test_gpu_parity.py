"""GPU (HIP, through the C ABI) against the FP64 CPU oracle on the same seeded
inputs.  Tolerances: relative L1 <= 1e-12 for FP64 runs and <= 1e-5 for FP32
values with FP64 positions; bit-exact where the method is exact (identity,
integer-cell translations); order histograms equal."""
import sys

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W
from tests.util import l1_rel, linf, oracle_problem, stored_values, tol

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


def gpu_run(B, torch, wl, nsteps=1, t0=0.0, kevery=1, **over):
    """Run nsteps GPU steps from wl's stored initial values; returns (fields as
    FP64 numpy, stats, status, grid)."""
    g = B.Grid.from_workload(wl, reconstruct_every=kevery, **over)
    fin = g.new_fields(stored_values(wl))
    out = g.advance(fin, t0, wl.dt, nsteps)
    rc, st = g.sync()
    res = [f.double().cpu().numpy() for f in out]
    return res, st, rc, g


def oracle_run(orc, wl, nsteps=1, t0=0.0, kevery=1, **kw):
    rc, fs, st = orc.run(oracle_problem(orc, wl, **kw), t0, wl.dt, nsteps,
                         stored_values(wl), kevery=kevery)
    return fs, st, rc


# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("m", [0, 1, 2])
@pytest.mark.parametrize("limiter", [False, True])
def test_identity_step_bitwise(B, torch, dim, prec, m, limiter):
    shape = (20, 24) if dim == 2 else (10, 12, 14)
    say("identity", dim, prec, m, limiter)
    g = np.random.Generator(np.random.PCG64(1))
    fs = [W.gaussian(shape, (0.4,) * dim, 0.15), W.disk(shape, (0.55,) * dim, 0.2),
          g.standard_normal(shape)]
    wl = W.uniform_translation(shape, [0.0] * dim, 0.1, fs, order_max=m, limiter=limiter,
                               value_prec=prec)
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=2)
    assert rc == 0 and st["search_fail"] == 0 and st["walked"] == 0
    for a, b in zip(out, stored_values(wl)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,shift", [((32, 16), (3, -2)), ((16, 32), (-7, 5)),
                                         ((8, 16, 16), (-5, 1, 2))])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_integer_translation_bitwise(B, torch, orc, shape, shift, prec):
    say("shift", shape, shift, prec)
    d = len(shape)
    dt = 0.125
    vel = [shift[a] / shape[d - 1 - a] / dt for a in range(d)]
    g = np.random.Generator(np.random.PCG64(2))
    fs = [W.disk(shape, (0.5,) * d, 0.3), g.standard_normal(shape)]
    for limiter in (False, True):
        wl = W.uniform_translation(shape, vel, dt, fs, limiter=limiter, value_prec=prec)
        out, st, rc, _ = gpu_run(B, torch, wl)
        assert rc == 0
        axes = tuple(range(d))[::-1]
        for a, b in zip(out, stored_values(wl)):
            assert np.array_equal(a, np.roll(b, shift, axis=axes))
        want, _, orc_rc = oracle_run(orc, wl)
        assert orc_rc == 0
        for a, b in zip(out, want):
            assert np.array_equal(a, b)


def _traj_cases():
    yield "uniform2d", W.uniform_translation((24, 20), [0.3, -0.2], 0.05, [np.zeros((24, 20))])
    yield "sbr", W.solid_body_gaussian(48, 100)
    yield "swirl", W.swirl_three_fields(40, value_prec="f64")  # large stage offsets
    yield "swirl256", W.swirl_three_fields(256, value_prec="f64")  # small offsets
    yield "deform3d", W.deform3d_slotted_sphere(16, nsteps=4)
    yield "deform3d64", W.deform3d_slotted_sphere(64, nsteps=4)
    w = W.fourier3d_three_fields(12, seed=3)
    yield "fourier3d", w
    w2 = W.serving_request(W.rng(5), 0, 0.0, sides=(64,)).workload
    w2.value_prec = "f64"
    yield "fourier2d", w2
    # Wave vectors outside the small-integer encoding (a component of 5 and a
    # fractional one): the modes take one cosine each.
    w3 = W.serving_request(W.rng(5), 0, 0.0, sides=(64,)).workload
    w3.value_prec = "f64"
    w3.velocity.modes = w3.velocity.modes.copy()
    w3.velocity.modes[0, :2] = (5.0, -1.0)
    w3.velocity.modes[1, :2] = (0.5, 2.0)
    yield "fourier2d_large_k", w3
    # Velocity given on the mesh (Z-spline interpolation of the samples).
    yield "gridded_swirl_z2", W.gridded(W.swirl_three_fields(40, value_prec="f64"), 2, t=0.4)
    yield "gridded_swirl_z0", W.gridded(W.swirl_three_fields(36, value_prec="f64"), 0, t=0.4)
    yield "gridded_fourier3d_z1", W.gridded(W.fourier3d_three_fields(12, seed=3), 1)


@pytest.mark.parametrize("name,wl", list(_traj_cases()))
@pytest.mark.parametrize("integrator", [0, 1])
def test_trajectories_match_oracle(B, torch, orc, name, wl, integrator):
    say("traj", name, integrator)
    wl.integrator = integrator
    g = B.Grid.from_workload(wl)
    t = 0.37
    for k in range(2):  # the second step continues from the stored displacement
        g.step(t + k * wl.dt, wl.dt)
    disp = g.displacement().cpu().numpy()
    prob = oracle_problem(orc, wl)
    want = orc.trajectories(prob, t, wl.dt)
    want = orc.trajectories(prob, t + wl.dt, wl.dt, want)
    assert np.abs(disp - want).max() < 1e-12, np.abs(disp - want).max()


def _step_cases():
    yield "sbr64", W.solid_body_gaussian(64, 100), 0.0
    yield "swirl_f64", W.swirl_three_fields(96, value_prec="f64"), 1.3
    yield "swirl_f32", W.swirl_three_fields(96, value_prec="f32"), 1.3
    yield "swirl_odd", W.swirl_three_fields(70, value_prec="f64"), 0.4
    w = W.serving_request(W.rng(7), 0, 0.0, sides=(128,)).workload
    w.fields = [f[:, :100].copy() for f in w.fields]  # ragged: 128 x 100
    w.shape = (128, 100)
    w.length = (1.0, 100 / 128)
    yield "fourier2d_ragged_f32", w, 0.0
    w = W.serving_request(W.rng(8), 0, 0.0, sides=(64,)).workload
    w.value_prec = "f64"
    w.order_max = 1
    yield "fourier2d_z1", w, 0.0
    yield "fourier3d_f64", W.fourier3d_three_fields(20, value_prec="f64"), 0.0
    yield "fourier3d_f32", W.fourier3d_three_fields(20, value_prec="f32"), 0.0
    yield "deform3d_f64", W.deform3d_slotted_sphere(24), 0.5
    yield "deform3d_f32", W.deform3d_slotted_sphere(24, value_prec="f32"), 0.5
    # Several full tiles (interior waves take the buffer-load gather) plus a
    # ragged edge tile in every axis.
    yield "fourier3d_f32_50", W.fourier3d_three_fields(50, value_prec="f32"), 0.0
    yield "deform3d_f64_42", W.deform3d_slotted_sphere(42), 1.0
    yield "gridded_swirl_f32", W.gridded(W.swirl_three_fields(96, value_prec="f32"), 2, t=1.3), 1.3
    yield "gridded_deform3d_f64", W.gridded(W.deform3d_slotted_sphere(24), 1, t=0.5), 0.5
    yield "burgers2d_f64", W.burgers(96), 0.0
    yield "burgers2d_f32", W.burgers(96, value_prec="f32"), 0.0
    yield "burgers3d_f64", W.burgers(24, dim=3), 0.0


@pytest.mark.parametrize("name,wl,t0", list(_step_cases()))
def test_single_step_parity(B, torch, orc, name, wl, t0):
    say("step", name, wl.shape, wl.value_prec)
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=1, t0=t0)
    want, ost, orc_rc = oracle_run(orc, wl, nsteps=1, t0=t0)
    assert rc == 0 and orc_rc == 0
    for f, (a, b) in enumerate(zip(out, want)):
        e = l1_rel(a, b)
        say("  field", f, "L1", e, "Linf", linf(a, b))
        assert e <= tol(wl), (f, e)
    assert st["order_hist"] == ost["order_hist"]
    assert st["search_fail"] == 0 and st["newton_fail"] == 0


@pytest.mark.parametrize("name,wl,nsteps", [
    ("sbr64_turn", W.solid_body_gaussian(64, 100), 100),
    ("swirl64_f64", W.swirl_three_fields(64, value_prec="f64"), 20),
    ("swirl64_f32", W.swirl_three_fields(64, value_prec="f32"), 20),
    ("fourier3d16_f64", W.fourier3d_three_fields(16, value_prec="f64"), 6),
    ("gridded_swirl64_f64", W.gridded(W.swirl_three_fields(64, value_prec="f64"), 2), 10),
    ("burgers2d64_f64", W.burgers(64), 40),
    ("burgers2d64_f32", W.burgers(64, value_prec="f32"), 40),
    ("burgers3d20_f64", W.burgers(20, dim=3), 8),
])
def test_multi_step_parity(B, torch, orc, name, wl, nsteps):
    say("run", name, nsteps)
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=nsteps)
    want, ost, orc_rc = oracle_run(orc, wl, nsteps=nsteps)
    assert rc == 0 and orc_rc == 0
    for f, (a, b) in enumerate(zip(out, want)):
        e = l1_rel(a, b)
        say("  field", f, "L1", e, "Linf", linf(a, b))
        assert e <= tol(wl), (f, e)


def test_reconstruct_every_two_steps(B, torch, orc):
    wl = W.swirl_three_fields(48, value_prec="f64")
    say("kevery 2")
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=6, kevery=2)
    want, ost, orc_rc = oracle_run(orc, wl, nsteps=6, kevery=2)
    assert rc == 0 and orc_rc == 0
    for a, b in zip(out, want):
        assert l1_rel(a, b) <= 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_minimum_grid_and_max_fields(B, torch, orc, dim):
    shape = (6,) * dim
    say("min grid", dim)
    g = np.random.Generator(np.random.PCG64(4))
    fs = [g.uniform(0, 1, shape) for _ in range(8)]
    wl = W.uniform_translation(shape, [0.31 / 6, -0.17 / 6, 0.09 / 6][:dim], 1.0, fs,
                               limiter=True)
    out, st, rc, _ = gpu_run(B, torch, wl)
    want, ost, orc_rc = oracle_run(orc, wl)
    assert rc == 0 and orc_rc == 0
    for a, b in zip(out, want):
        assert l1_rel(a, b) <= 1e-12
    assert st["order_hist"] == ost["order_hist"]


def test_box_too_large_for_lds_takes_global_path(B, torch, orc):
    """Eight FP64 fields do not fit a tile's staging box in LDS: every tile
    takes the global-memory path, with the same results."""
    wl = W.swirl_three_fields(64, value_prec="f64")
    g = np.random.Generator(np.random.PCG64(6))
    wl.fields = wl.fields + [g.uniform(0, 1, wl.shape) for _ in range(5)]
    say("8 fields f64")
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=2, t0=0.3)
    want, ost, orc_rc = oracle_run(orc, wl, nsteps=2, t0=0.3)
    assert rc == 0 and orc_rc == 0
    for a, b in zip(out, want):
        assert l1_rel(a, b) <= 1e-12


def test_search_failure_is_reported_like_the_oracle(B, torch, orc):
    """A folded lattice (solid-body rotation with a huge step, corners of the
    periodic box) with the fallback scan disabled: the same nodes fail on both
    sides, sl_sync reports SL_ESEARCH, failed nodes hold NaN."""
    wl = W.solid_body_gaussian(32, 12)
    say("search failure")
    over = dict(scan_radius=0, walk_max=6)
    out, st, rc, _ = gpu_run(B, torch, wl, **over)
    want, ost, orc_rc = oracle_run(orc, wl, scan_radius=0, walk_max=6)
    assert orc_rc == orc.ESEARCH and ost["search_fail"] > 0
    assert rc == B.SL_ESEARCH
    assert st["search_fail"] == ost["search_fail"]
    assert np.array_equal(np.isnan(out[0]), np.isnan(want[0]))
    ok = ~np.isnan(want[0])
    assert l1_rel(out[0][ok], want[0][ok]) <= 1e-12


@pytest.mark.parametrize("theta", [0.25, 0.1])
def test_jump_flags_at_ties_fp32(B, torch, orc, theta):
    """FP32 fields built so that the jump criterion sits at or within a few
    ulps of its threshold at most nodes: the GPU's screened FP32 evaluation
    must take exactly the oracle's FP64 decision everywhere (same orders,
    same values)."""
    g = np.random.Generator(np.random.PCG64(12))
    n = 64
    # Along x, triples (a, 0, c) with c - 2*0 + a = theta * max(|c|, |a|)
    # exactly in reals, then nudged by -2..2 ulps.
    # Constant along y, so only the x test can fire at the middle nodes.
    c = g.uniform(0.5, 2.0, n).astype(np.float32)
    a = (np.float32(theta) * c - c).astype(np.float32)
    row = np.zeros(n, np.float32)
    row[0::3] = a[0::3]
    row[2::3] = c[2::3]
    ulps = g.integers(-2, 3, n).astype(np.int32)
    row = (row.view(np.int32) + np.where(row != 0, ulps, 0)).view(np.float32)
    f = np.tile(row, (n, 1))
    f2 = np.ascontiguousarray(f.T)
    wl = W.uniform_translation((n, n), [0.37 / n, -0.21 / n], 1.0,
                               [f.astype(np.float64), f2.astype(np.float64)],
                               limiter=True, value_prec="f32")
    wl.theta = theta
    say("ties", theta)
    out, st, rc, _ = gpu_run(B, torch, wl)
    want, ost, orc_rc = oracle_run(orc, wl)
    assert rc == 0 and orc_rc == 0
    assert st["order_hist"] == ost["order_hist"]
    for a_, b_ in zip(out, want):
        assert np.abs(a_ - b_).max() <= 1e-5 * np.abs(b_).max()


def _edge_nodes(field, z_lo, z_hi, planes):
    """Linear indices of nodes where a 0/1 field changes along x, taken from a
    few planes (3-D, array axis 0 in [z_lo, z_hi)) or rows (2-D) through the
    body, without a pass over the whole grid."""
    nx = field.shape[-1]
    out = []
    for z in np.linspace(z_lo, z_hi - 1, planes).astype(np.int64):
        sl = np.asarray(field[z])
        idx = np.nonzero(np.diff(sl, axis=-1, append=sl[..., :1]) != 0)
        lin = idx[-1] + (idx[0] * nx if sl.ndim == 2 else 0)
        out.append(lin + z * sl.size)
    return np.concatenate(out)


def _large_workload(which):
    """Grids above 2^28 nodes, where one field's or one displacement
    component's bytes exceed the 31-bit buffer offsets and the kernels take
    their plain-pointer paths: 650^3 FP64 (ragged tiles in every axis),
    1024 x 1024 x 1023 with FP32 values (the largest grid a descriptor
    accepts, 2^30 - 2^20 nodes) and a 16400^2 swirl in FP64."""
    if which == "deform650_f64":
        return W.deform3d_slotted_sphere(650), 0.7
    if which == "deform_max_f32":
        shape = (1023, 1024, 1024)
        fs = [W.slotted_disk(shape, (0.35, 0.35, 0.35), 0.15, 0.05, 0.25).astype(np.float32)]
        return W.Workload("deform3d_max_f32", shape, (1.0, 1.0, 1.0), fs,
                          W.Velocity(W.VEL_DEFORM3D, [3.0, 1.0]), dt=1.5 / 1024, nsteps=1,
                          order_max=2, limiter=True, value_prec="f32"), 0.7
    shape = (16400, 16400)
    fs = [W.slotted_disk(shape, (0.5, 0.75), 0.15, 0.05, 0.25)]
    return W.Workload("swirl2d_16400_f64", shape, (1.0, 1.0), fs,
                      W.Velocity(W.VEL_SWIRL2D, [5.0, 1.0]), dt=4.0 / 16400, nsteps=1,
                      order_max=2, limiter=True, value_prec="f64"), 1.1


@pytest.mark.parametrize("which", ["deform650_f64", "deform_max_f32", "swirl16400_f64"])
def test_grids_beyond_buffer_offsets_sampled(B, torch, orc, which):
    """One step on grids whose fields or displacement components exceed 2^31
    bytes (the plain-pointer paths of the element solve and the gathers, and
    32-bit node indices up to the largest grid), checked at sampled nodes
    (random ones and nodes on the body's edge) that the oracle evaluates one
    by one; the sample is gathered on the device."""
    wl, t0 = _large_workload(which)
    say("beyond buffer offsets", which, wl.shape)
    vals = stored_values(wl)
    g = B.Grid.from_workload(wl)
    out = g.advance(g.new_fields(vals), t0, wl.dt, 1)
    rc, st = g.sync()
    assert rc == 0 and st["search_fail"] == 0 and st["newton_fail"] == 0
    assert st["nodes"] == wl.nodes
    gen = np.random.Generator(np.random.PCG64(13))
    nz = wl.shape[0]
    lo, hi = (int(0.22 * nz), int(0.48 * nz)) if wl.dim == 3 else (int(0.62 * nz), int(0.88 * nz))
    edge = _edge_nodes(wl.fields[0], lo, hi, 12 if wl.dim == 3 else 64)
    sample = np.unique(np.concatenate([gen.integers(0, wl.nodes, 2000),
                                       gen.choice(edge, 1000)]))
    idx = torch.as_tensor(sample, device=out[0].device)
    got = out[0].reshape(-1)[idx].double().cpu().numpy()
    del out
    rc2, ref, _ = orc.step_sampled(oracle_problem(orc, wl), t0, wl.dt, vals, sample)
    assert rc2 == 0
    err = np.abs(got - ref[:, 0]).max()
    say("  max abs err", err, "at", sample.size, "nodes")
    assert err <= (1e-5 if wl.value_prec == "f32" else 1e-12) * max(1.0, np.abs(ref[:, 0]).max())


@pytest.mark.parametrize("name,wl", [
    ("swirl96_f32", W.swirl_three_fields(96, value_prec="f32")),
    ("fourier3d_28_f32", W.fourier3d_three_fields(28, value_prec="f32")),
    ("deform3d_24_f64", W.deform3d_slotted_sphere(24)),
    ("fourier2d_96_f32", W.serving_request(W.rng(7), 0, 0.0, sides=(96,)).workload),
])
def test_per_call_path_equals_advance(B, torch, name, wl):
    """sl_step / sl_reconstruct called one by one give the same bits as
    sl_advance (where each reconstruction also integrates the next step's
    trajectories, starting from the per-axis sin/cos table where the velocity
    family has one), and kernel events do not change results."""
    a, _, _, _ = gpu_run(B, torch, wl, nsteps=4, t0=0.6)
    g = B.Grid.from_workload(wl)
    g.profile(True)
    x = g.new_fields(stored_values(wl))
    y = g.new_fields()
    for s in range(4):
        g.step(0.6 + s * wl.dt, wl.dt)
        g.reconstruct(x, y)
        x, y = y, x
    prof = g.profile_read()
    assert prof["recon_launches"] == 4 and prof["traj_launches"] == 4
    assert prof["recon_ms"] > 0 and prof["traj_ms"] > 0
    rc, _ = g.sync()
    assert rc == 0
    for p, q in zip(a, x):
        assert np.array_equal(p, q.double().cpu().numpy())


def test_repeatable_bitwise(B, torch):
    wl = W.swirl_three_fields(128, value_prec="f32")
    a, _, _, _ = gpu_run(B, torch, wl, nsteps=3, t0=0.2)
    b, _, _, _ = gpu_run(B, torch, wl, nsteps=3, t0=0.2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_full_size_swirl_sampled(B, torch, orc):
    """The 1024^2 three-field swirl (FP32 values, FP64 positions, limiter on):
    one full GPU step, checked at sampled nodes (random ones and every node
    near the slotted-disc edge) that the oracle evaluates one by one."""
    wl = W.swirl_three_fields(1024, value_prec="f32")
    t0 = 1.1
    say("full size swirl 1024^2")
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=1, t0=t0)
    assert rc == 0
    g = np.random.Generator(np.random.PCG64(9))
    n = wl.nodes
    edge = np.nonzero(np.abs(np.diff(wl.fields[0].ravel(), append=0.0)) > 0)[0]
    sample = np.unique(np.concatenate([g.integers(0, n, 3000), g.choice(edge, 1500)]))
    rc2, vals, ost = orc.step_sampled(oracle_problem(orc, wl), t0, wl.dt,
                                      stored_values(wl), sample)
    assert rc2 == 0
    for f in range(wl.nfields):
        got = out[f].ravel()[sample]
        err = np.abs(got - vals[:, f]).max()
        say("  field", f, "max abs err", err)
        assert err <= 1e-5 * max(1.0, np.abs(vals[:, f]).max())


@pytest.mark.parametrize("which", ["fourier256_f32", "deform512_f64"])
def test_full_size_3d_sampled(B, torch, orc, which):
    """The 3-D workloads at full size (256^3 three fields FP32, 512^3 one
    field FP64): one GPU step, checked at sampled nodes (random ones and
    nodes next to the slotted sphere's surface) that the oracle evaluates one
    by one."""
    if which == "fourier256_f32":
        wl, t0 = W.fourier3d_three_fields(256, value_prec="f32"), 0.0
    else:
        wl, t0 = W.deform3d_slotted_sphere(512), 0.7
    say("full size", which)
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=1, t0=t0)
    assert rc == 0 and st["search_fail"] == 0 and st["newton_fail"] == 0
    g = np.random.Generator(np.random.PCG64(11))
    n = wl.nodes
    edge = np.nonzero(np.abs(np.diff(wl.fields[0].ravel(), append=0.0)) > 0)[0]
    sample = np.unique(np.concatenate([g.integers(0, n, 2000), g.choice(edge, 1000)]))
    rc2, vals, ost = orc.step_sampled(oracle_problem(orc, wl), t0, wl.dt,
                                      stored_values(wl), sample)
    assert rc2 == 0
    rel = 1e-5 if wl.value_prec == "f32" else 1e-12
    for f in range(wl.nfields):
        got = out[f].ravel()[sample]
        err = np.abs(got - vals[:, f]).max()
        say("  field", f, "max abs err", err)
        assert err <= rel * max(1.0, np.abs(vals[:, f]).max())


@pytest.mark.parametrize("name,wl", [
    ("swirl96_f32", W.swirl_three_fields(96, value_prec="f32")),
    ("swirl96_f64", W.swirl_three_fields(96, value_prec="f64")),
    ("swirl70_f64", W.swirl_three_fields(70, value_prec="f64")),
    ("swirl1280_f32", W.swirl_three_fields(1280, value_prec="f32")),
])
def test_2d_limiter_paths_agree_bitwise(B, torch, name, wl):
    """2-D grids take the limiter flags either inside the reconstruction
    tiles or from the separate order-word pass (quad kernels when rows are a
    multiple of 4: flags and x window in one launch for rows of up to 256
    quads, as at 96, in two beyond, as at 1280; scalar kernels otherwise, as
    at 70); both give the same orders, so the results are bitwise equal."""
    outs = []
    for where in (B.SL_LIMITER_IN_TILES, B.SL_LIMITER_ORDER_WORDS):
        out, st, rc, _ = gpu_run(B, torch, wl, nsteps=3, t0=1.1, limiter_pass=where)
        assert rc == 0
        outs.append((out, st["order_hist"]))
    (a, ha), (b, hb) = outs
    assert ha == hb
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name,wl", [
    ("swirl", W.swirl_three_fields(64, value_prec="f64")),
    ("burgers", W.burgers(64)),
    # The second lattice step starts ~4 cells out, so its stage points leave
    # the gridded kernel's LDS box and take its global path.
    ("gridded", W.gridded(W.swirl_three_fields(64, value_prec="f64"), 2, t=0.7)),
])
def test_reconstruct_every_two_steps_carried_and_prescribed(B, torch, orc, name, wl):
    """Two lattice steps per reconstruction (K = 2): prescribed velocities
    continue the RK integration, a carried velocity continues the straight
    line of the last reset."""
    out, st, rc, _ = gpu_run(B, torch, wl, nsteps=8, kevery=2)
    want, ost, orc_rc = oracle_run(orc, wl, nsteps=8, kevery=2)
    assert rc == 0 and orc_rc == 0
    for f, (a, b) in enumerate(zip(out, want)):
        e = l1_rel(a, b)
        say("  field", f, "L1", e)
        assert e <= tol(wl), (f, e)

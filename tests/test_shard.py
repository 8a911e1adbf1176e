"""One GPU's share of a larger grid: a shard is a grid whose node 0 sits at a
given index of the whole periodic lattice (`offset`), with halo planes around
the nodes it owns.  Its lattice moves exactly as the same nodes of the whole
grid, so when the halo holds the neighbours' values (refreshed between steps,
as a halo exchange would) the owned nodes' results equal the whole grid's
bit for bit.  CPU checks use the oracle; GPU checks compare the shard with the
whole-grid GPU run."""
import ctypes as C

import numpy as np
import pytest

from paper_1410_2817_amd import workloads as W
from tests.util import oracle_problem, stored_values

HALO = 8  # > largest displacement (4 cells at CFL 4) + stencil half-width + walk margin


def _slab(a, axis, lo, hi):
    """Periodic slab [lo, hi) of array a along axis."""
    idx = np.arange(lo, hi) % a.shape[axis]
    return np.take(a, idx, axis=axis)


def _cases():
    # (name, whole-grid workload, owned range [lo, hi) along the slowest array
    # axis (y in 2-D, z in 3-D), bitwise?)  A shard that wraps around the
    # periodic boundary evaluates the velocity at x + 1 where the whole grid
    # uses x: equal in exact arithmetic, not in rounding.
    yield "swirl2d", W.swirl_three_fields(128, value_prec="f64"), (40, 72), True
    yield "swirl2d_f32", W.swirl_three_fields(128, value_prec="f32"), (64, 80), True
    yield "swirl2d_wrapped", W.swirl_three_fields(128, value_prec="f64"), (120, 136), False
    yield "deform3d", W.deform3d_slotted_sphere(48), (16, 32), True


def _shard_problem(orc, wl, axis, lo, hi):
    shape = list(wl.shape)
    shape[axis] = hi - lo + 2 * HALO
    off = [0] * wl.dim
    off[axis] = lo - HALO
    ln = list(wl.length)
    ln[axis] = wl.length[axis] * shape[axis] / wl.shape[axis]
    return shape, off, ln


# --------------------------------------------------------------------------
# CPU: the oracle

def test_oracle_shard_trajectories_are_the_whole_grids(orc):
    wl = W.deform3d_slotted_sphere(32)
    shape, off, ln = _shard_problem(orc, wl, 0, 10, 20)
    whole = orc.trajectories(oracle_problem(orc, wl), 0.4, wl.dt)
    p = orc.Problem(shape, 1, ln, vel_kind=wl.velocity.kind, vp=wl.velocity.padded_params(),
                    offset=off)
    part = orc.trajectories(p, 0.4, wl.dt)
    assert np.array_equal(part, _slab(whole, 1, off[0], off[0] + shape[0]))


def test_oracle_shard_step_matches_the_whole_grid_inside(orc):
    wl = W.swirl_three_fields(96, value_prec="f64")
    lo, hi = 30, 50
    shape, off, ln = _shard_problem(orc, wl, 0, lo, hi)
    t0 = 1.1
    rc, full, _ = orc.run(oracle_problem(orc, wl), t0, wl.dt, 1, stored_values(wl))
    assert rc == 0
    p = orc.Problem(shape, wl.nfields, ln, order_max=2, limiter=wl.limiter, theta=wl.theta,
                    vel_kind=wl.velocity.kind, vp=wl.velocity.padded_params(), offset=off)
    init = [_slab(f, 0, off[0], off[0] + shape[0]) for f in stored_values(wl)]
    rc, part, _ = orc.run(p, t0, wl.dt, 1, init)
    assert rc == 0
    for a, b in zip(part, full):
        assert np.array_equal(a[HALO:-HALO], b[lo:hi])


def test_descriptor_offsets_are_validated():
    from paper_1410_2817_amd import binding as B
    lib = B.load()

    def create(**kw):
        d, _ = B.make_desc(kw.pop("shape", (32, 32)), kw.pop("nfields", 3), **kw)
        h = C.c_void_p()
        rc = lib.sl_create_grid(C.byref(d), C.byref(h))
        if h.value:
            lib.sl_destroy_grid(h)
        return rc

    assert create(offset=(5, -7)) == B.SL_OK
    assert create(offset=(1 << 30, 0)) == B.SL_EINVAL
    assert create(offset=(3, 0), vel_kind=5, vel_params=[2.0]) == B.SL_EINVAL
    assert create(offset=(3, 0), vel_kind=6, integrator=B.SL_RK3_WILLIAMSON,
                  source=B.SL_SRC_SHALLOW_WATER, source_p=[0, 1, 0.5, 0]) == B.SL_EINVAL


# --------------------------------------------------------------------------
# GPU: a shard against the whole grid, with the halo refreshed between steps

@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.fail("no GPU visible")
    return T


@pytest.mark.gpu
@pytest.mark.parametrize("name,wl,rng,bitwise", list(_cases()))
def test_gpu_shard_matches_the_whole_grid(torch, orc, name, wl, rng, bitwise):
    from paper_1410_2817_amd import binding as B
    lo, hi = rng
    shape, off, ln = _shard_problem(orc, wl, 0, lo, hi)
    full = B.Grid.from_workload(wl)
    shard = B.Grid(shape, wl.nfields, length=ln, value_prec=wl.value_prec,
                   order_max=wl.order_max, limiter=wl.limiter, theta=wl.theta,
                   integrator=wl.integrator, vel_kind=wl.velocity.kind,
                   vel_params=wl.velocity.padded_params(), modes=wl.velocity.modes, offset=off)
    st = stored_values(wl)
    f_full = full.new_fields(st)
    f_part = shard.new_fields([_slab(a, 0, off[0], off[0] + shape[0]) for a in st])
    t0 = 0.7
    for k in range(4):
        t = t0 + k * wl.dt
        f_full = full.advance(f_full, t, wl.dt, 1)
        f_part = shard.advance(f_part, t, wl.dt, 1)
        whole = [f.double().cpu().numpy() for f in f_full]
        part = [f.double().cpu().numpy() for f in f_part]
        for a, b in zip(part, whole):
            got, want = a[HALO:-HALO], _slab(b, 0, lo, hi)
            assert np.isfinite(got).all(), (name, k)
            if bitwise:
                assert np.array_equal(got, want), (name, k)
            else:
                assert np.abs(got - want).sum() <= 1e-12 * np.abs(want).sum(), (name, k)
        # halo exchange: the shard's halo planes from the whole grid
        f_part = shard.new_fields([_slab(b, 0, off[0], off[0] + shape[0]) for b in whole])
    rc1, _ = full.sync()
    rc2, _ = shard.sync()
    # The shard also reconstructs its halo, whose outermost nodes may not find a
    # host element across the shard's own periodic seam (planes 0 and n-1 are
    # not neighbours in the whole grid); its owned nodes never reach the seam.
    assert rc1 == 0 and rc2 in (0, B.SL_ESEARCH)

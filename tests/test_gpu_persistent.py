"""The persistent batched form and the block sizes through the C-ABI: a
batch whose substeps run as one cooperative launch gives results bitwise
equal to the graph of launches, to each instance run alone and (FP64) to the
oracle; block sizes of the column and vertex kernels are result-neutral; the
autotuner searches them."""
import numpy as np
import pytest

import oracle
from paper_2511_02021_amd.inputs import case as CS

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def _cases():
    # uneven sizes and level counts, a one-block grid among them
    return [CS.make_case(3, 20, z_top=30000.0, noise_seed=[0, 4, 0], dt=300.0),
            CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 4, 1],
                         noise_seed=[0, 4, 1], dt=150.0),
            CS.make_case(0, 2, z_top=30000.0, noise_seed=[0, 4, 3], dt=300.0),
            CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 4, 2],
                         noise_seed=[0, 4, 2], dt=300.0)]


def _batch_states(cases, precision, persistent, tiles=None, steps=3, blocks_per_cu=0):
    nhdc = _nhdc()
    ds = [nhdc.Dycore(c, precision=precision) for c in cases]
    b = nhdc.Batch(ds)
    if tiles:
        b.set_tiles(*tiles)
    if persistent:
        print(f"persistent batch {precision} tiles={tiles}", flush=True)
        b.set_persistent(True, blocks_per_cu)
        assert b.persistent_grid > 0
    b.step([c.dt for c in cases], 5, nsteps=steps)
    out = [(d.get_state(), d.mass_flux()) for d in ds]
    b.close()
    for d in ds:
        d.close()
    return out


@pytest.mark.parametrize("precision,tiles,per_cu", [("fp64", None, 0), ("fp64", (16, 8, 16), 0),
                                                    ("mixed", None, 0), ("fp64", None, 1)])
def test_persistent_batch_equals_graph_of_launches(precision, tiles, per_cu):
    cases = _cases()
    ref = _batch_states(cases, precision, False, tiles)
    got = _batch_states(cases, precision, True, tiles, blocks_per_cu=per_cu)
    for i, ((s, f), (rs, rf)) in enumerate(zip(got, ref)):
        for fld in FIELDS:
            assert np.array_equal(s[fld], rs[fld]), (i, fld)
        assert np.array_equal(f[0], rf[0]) and np.array_equal(f[1], rf[1]), i
    if precision == "fp64" and tiles is None and per_cu == 0:
        for c, (s, _) in zip(cases, got):  # and the oracle
            m = oracle.Model(c)
            for _ in range(3):
                m.step(c.dt, 5)
            o = m.state()
            for fld in FIELDS:
                assert np.array_equal(s[fld], o[fld]), (c.grid.k, fld)


def test_persistent_batch_with_every_option():
    """Upwind, damped (fourth-order damping, sponge, diffusion) and tracer
    instances next to plain ones: the persistent kernel's upwind, sponge and
    damping builds, and the once-per-step launches around it."""
    base = _cases()
    cases = [CS.with_params(base[0], upwind=1), CS.with_damping(base[1], sponge_base=20000.0),
             CS.with_tracers(base[3]), base[2]]
    nhdc = _nhdc()
    res = {}
    for persistent in (False, True):
        ds = [nhdc.Dycore(c) for c in cases]
        b = nhdc.Batch(ds)
        if persistent:
            b.set_persistent(True)
        b.step([c.dt for c in cases], 5, nsteps=2)
        res[persistent] = [(d.get_state(), d.get_tracers()) for d in ds]
        b.close()
        for d in ds:
            d.close()
    for i, ((s, q), (rs, rq)) in enumerate(zip(res[True], res[False])):
        for fld in FIELDS:
            assert np.array_equal(s[fld], rs[fld]), (i, fld)
        assert np.array_equal(q, rq), i


def test_persistent_refused_for_other_numberings():
    nhdc = _nhdc()
    c = CS.config_case(2, k=4, n_lev=10, order="random")
    d = nhdc.Dycore(c)
    b = nhdc.Batch([d])
    with pytest.raises(nhdc.NhdcError) as e:
        b.set_persistent(True)
    assert e.value.code == -1
    b.close()
    d.close()


@pytest.mark.parametrize("column,vertex,waves", [(64, 64, 3), (128, 256, 0), (256, 128, 2),
                                                (64, 128, 0), (256, 256, 0)])
def test_block_sizes_are_result_neutral(column, vertex, waves):
    nhdc = _nhdc()
    c = CS.config_case(2, k=4, n_lev=30)
    ref = nhdc.Dycore(c)
    d = nhdc.Dycore(c)
    d.set_block_sizes(column, vertex, waves)
    for _ in range(3):
        ref.step(c.dt, 5)
        d.step(c.dt, 5)
    s, r = d.get_state(), ref.get_state()
    for f in FIELDS:
        assert np.array_equal(s[f], r[f]), (column, vertex, waves, f)
    with pytest.raises(nhdc.NhdcError):
        d.set_block_sizes(96, 256)
    with pytest.raises(nhdc.NhdcError):
        d.set_block_sizes(256, 256, 1)
    d.close()
    ref.close()


def test_persistent_batch_autotune_restores_state(tmp_path):
    nhdc = _nhdc()
    cases = _cases()
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    b.set_persistent(True)
    before = [d.get_state() for d in ds]
    best = b.autotune([c.dt for c in cases], 5, cache_path=str(tmp_path / "t.json"))
    assert all(t in (0, 48, 32, 16, 8, 4) for t in best[:3]) and best[6] > 0
    assert "persistent" in open(tmp_path / "t.json").read()
    for d, s0 in zip(ds, before):
        s = d.get_state()
        for f in FIELDS:
            assert np.array_equal(s[f], s0[f]), f
    b.close()
    for d in ds:
        d.close()

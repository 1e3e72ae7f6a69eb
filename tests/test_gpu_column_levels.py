"""The level-parallel column build through the C-ABI: with the levels of each
column shared among lanes and the Thomas factors in LDS, every form gives the
streaming build's results to the bit (and so, in FP64, the oracle's), over
ragged level counts, the smallest grids, the library's 256 levels, every
option and batches of uneven instances."""
import numpy as np
import pytest

import oracle
from paper_2511_02021_amd.inputs import case as CS

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def _run(case, mode, precision="fp64", steps=3, tracers=False):
    nhdc = _nhdc()
    print(f"column mode {mode} {precision} R2B{case.grid.k}x{case.n_lev}", flush=True)
    d = nhdc.Dycore(case, precision=precision)
    d.set_column_mode(mode)
    for _ in range(steps):
        d.step(case.dt, case.nsub)
    out = (d.get_state(), d.mass_flux(), d.get_tracers() if tracers else None)
    d.close()
    return out


def _equal(a, b, tag):
    (s, f, q), (rs, rf, rq) = a, b
    for fld in FIELDS:
        assert np.array_equal(s[fld], rs[fld]), (tag, fld)
    assert np.array_equal(f[0], rf[0]) and np.array_equal(f[1], rf[1]), tag
    if q is not None:
        assert np.array_equal(q, rq), tag


# level counts: one level per lane group and empty groups (7), a ragged last
# group (45), the paper's 90, past the 16-column width (230), the maximum (256)
CASES = [
    ("r2b3x20 flat", lambda: CS.make_case(3, 20, z_top=30000.0, noise_seed=[0, 7, 0], dt=300.0)),
    ("r2b4x30 terrain", lambda: CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 1],
                                             noise_seed=[0, 7, 1], dt=150.0)),
    ("r2b0x2", lambda: CS.make_case(0, 2, z_top=30000.0, noise_seed=[0, 7, 2], dt=300.0)),
    ("r2b2x7", lambda: CS.make_case(2, 7, z_top=30000.0, terrain_seed=[1, 7, 3], noise_seed=[0, 7, 3],
                                    dt=300.0)),
    ("r2b3x45", lambda: CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 4],
                                     noise_seed=[0, 7, 4], dt=300.0)),
    ("r2b3x90", lambda: CS.config_case(2, k=3)),
    ("r2b1x230", lambda: CS.make_case(1, 230, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 5],
                                      noise_seed=[0, 7, 5], dt=300.0)),
    ("r2b0x256", lambda: CS.make_case(0, 256, z_top=75000.0, stretch=1.6, noise_seed=[0, 7, 6],
                                      dt=300.0)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_levels_build_equals_streaming_build_fp64(name, make):
    c = make()
    ref = _run(c, 0)
    got = _run(c, 1)
    _equal(got, ref, name)
    if c.grid.n_cells * c.n_lev <= 20480 * 30:  # and the oracle, where it is quick
        m = oracle.Model(c)
        for _ in range(3):
            m.step(c.dt, c.nsub)
        o = m.state()
        for fld in FIELDS:
            assert np.array_equal(got[0][fld], o[fld]), (name, fld)


@pytest.mark.parametrize("precision", ["mixed", "mixed_vn32"])
def test_levels_build_equals_streaming_build_mixed(precision):
    # the column is FP64 and formed without contraction in every form
    c = CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 1], noise_seed=[0, 7, 1],
                     dt=150.0)
    _equal(_run(c, 1, precision), _run(c, 0, precision), precision)


@pytest.mark.parametrize("option", ["upwind", "damped", "tracers"])
def test_levels_build_with_options(option):
    base = CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 4], noise_seed=[0, 7, 4],
                        dt=300.0)
    c = {"upwind": lambda: CS.with_params(base, upwind=1),
         "damped": lambda: CS.with_damping(base, sponge_base=30000.0),
         "tracers": lambda: CS.with_tracers(base)}[option]()
    tr = option == "tracers"
    _equal(_run(c, 1, tracers=tr), _run(c, 0, tracers=tr), option)


def test_levels_build_in_a_batch():
    """Uneven instances (2 to 45 levels) in one launch per kernel: each equal
    to the instance run alone with the streaming build."""
    nhdc = _nhdc()
    cases = [CS.make_case(3, 20, z_top=30000.0, noise_seed=[0, 7, 0], dt=300.0),
             CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 1], noise_seed=[0, 7, 1],
                          dt=150.0),
             CS.make_case(0, 2, z_top=30000.0, noise_seed=[0, 7, 2], dt=300.0),
             CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 4], noise_seed=[0, 7, 4],
                          dt=300.0)]
    refs = [_run(c, 0) for c in cases]
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    b.step([c.dt for c in cases], 5)  # a graph with the streaming column first
    b.set_column_mode(1)             # then re-captured with the levels build
    for d, c in zip(ds, cases):      # restart from the initial states
        d.init_state(c.vn, c.w, c.rho, c.pi, c.theta_v)
    print("batch with the levels build", flush=True)
    b.step([c.dt for c in cases], 5, nsteps=3)
    got = [(d.get_state(), d.mass_flux(), None) for d in ds]
    b.close()
    for d in ds:
        d.close()
    for i, (g, r) in enumerate(zip(got, refs)):
        _equal(g, r, i)


def test_column_mode_argument_checks():
    nhdc = _nhdc()
    c = CS.make_case(0, 2, z_top=30000.0, noise_seed=[0, 7, 2], dt=300.0)
    d = nhdc.Dycore(c)
    for bad in (-1, 2):
        with pytest.raises(nhdc.NhdcError) as e:
            d.set_column_mode(bad)
        assert e.value.code == -1
    b = nhdc.Batch([d])
    with pytest.raises(nhdc.NhdcError):
        b.set_column_mode(3)
    b.close()
    d.close()


@pytest.mark.parametrize("k,n_lev,expect", [(3, 90, (4, 4, 4, 1)), (4, 90, (8, 4, 8, 1)),
                                            (5, 90, (32, 16, 48, 0, 64)), (6, 30, (0, 0, 0, 0, 256))])
def test_starting_shapes_by_share_size(k, n_lev, expect):
    """Each marching kind starts with the largest level tile giving at least
    1024 blocks; the level-parallel column up to 40960 cells, else the
    streaming column in blocks of 64 lanes while it has fewer than 1024
    blocks of 256."""
    nhdc = _nhdc()
    c = CS.make_case(k, n_lev, z_top=75000.0, stretch=1.6, noise_seed=[0, 7, 8], dt=90.0)
    d = nhdc.Dycore(c)
    s = d.shapes_in_use
    assert (s[0], s[1], s[2], s[6]) == expect[:4], s
    if len(expect) > 4:
        assert s[3] == expect[4], s
    d.set_column_mode(1 - s[6])
    d.set_tiles(16, 16, 16)
    assert d.shapes_in_use[:3] == (16, 16, 16) and d.shapes_in_use[6] == 1 - s[6]
    b = nhdc.Batch([d])
    assert b.shapes_in_use[:3] == (s[0], s[1], s[2]) and b.shapes_in_use[6] == s[6]  # by the batch's size
    b.close()
    d.close()

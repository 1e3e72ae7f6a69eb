"""Edge cases of the HIP path through the C-ABI: the smallest grids (a single
ragged block), the fewest and the most levels the library takes, substep
counts, extreme level tiles, a batch at its instance limit, and the
properties that hold at the largest benchmark sizes where the oracle cannot
follow.  FP64 results are compared with the oracle (or with the same
instance run alone) bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2511_02021_amd.inputs import case as CS

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def _case(k, n_lev, tag=0, dt=None):
    deep = n_lev > 60
    return CS.make_case(k, n_lev, z_top=75000.0 if deep else 30000.0, stretch=1.6 if deep else 1.0,
                        terrain_seed=[9, k, n_lev, tag], noise_seed=[8, k, n_lev, tag],
                        dt=dt if dt is not None else 300.0 / (k + 1))


def _gpu(case, steps, nsub=5, tiles=None):
    d = _nhdc().Dycore(case)
    if tiles:
        d.set_tiles(*tiles)
    for _ in range(steps):
        d.step(case.dt, nsub)
    s, f = d.get_state(), d.mass_flux()
    d.close()
    return s, f


def _oracle(case, steps, nsub=5):
    m = oracle.Model(case)
    for _ in range(steps):
        m.step(case.dt, nsub)
    return m.state(), m.flux()


def _same(a, b, label):
    bad = {f: int(np.count_nonzero(a[f] != b[f])) for f in FIELDS}
    print(label, "differing entries", bad, flush=True)
    assert not any(bad.values()), (label, bad)


@pytest.mark.parametrize("k,n_lev", [(0, 2), (1, 3), (2, 7), (1, 256)])
def test_small_ragged_and_deep_grids_bitwise(k, n_lev):
    """R2B0 (80 cells: one partial block per kind), R2B1/R2B2 with ragged
    tails, the minimum of two levels and the library's maximum of 256."""
    c = _case(k, n_lev)
    gs, gf = _gpu(c, 3)
    os_, of = _oracle(c, 3)
    _same(gs, os_, f"R2B{k}x{n_lev}")
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])


@pytest.mark.parametrize("terrain,z_top", [(None, 30000.0), ([5, 1], 30000.0), ([5, 2], 12000.0),
                                           ([5, 3], 16500.0)])
def test_flat_top_regimes_bitwise(terrain, z_top):
    """The kernels read a neighbour's height without a gather at the leading
    half levels where every column has the same height.  Flat terrain (every
    level flat), terrain below a flat top, terrain reaching the lid (no flat
    level) and a lid just above the top of the terrain-following layer: each
    bitwise equal to the oracle, upwind and damping options included."""
    c = CS.make_case(3, 20, z_top=z_top, terrain_seed=terrain, noise_seed=[8, 3, 20, int(z_top)],
                     dt=100.0)
    c = CS.with_damping(CS.with_params(c, upwind=1))
    gs, gf = _gpu(c, 3)
    os_, of = _oracle(c, 3)
    _same(gs, os_, f"terrain={terrain} z_top={z_top}")
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])


@pytest.mark.parametrize("nsub", [1, 2, 3, 7])
def test_substep_counts_bitwise(nsub):
    c = _case(2, 10, tag=nsub)
    gs, gf = _gpu(c, 2, nsub=nsub)
    os_, of = _oracle(c, 2, nsub=nsub)
    _same(gs, os_, f"nsub={nsub}")
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])


def test_extreme_level_tiles_are_result_neutral():
    c = _case(3, 20)
    ref, rf = _gpu(c, 2)
    for tiles in ((1, 1, 1), (300, 300, 300), (3, 19, 2), (20, 21, 1)):
        s, f = _gpu(c, 2, tiles=tiles)
        _same(s, ref, f"tiles {tiles}")
        assert np.array_equal(f[0], rf[0]) and np.array_equal(f[1], rf[1])


def test_batch_at_the_instance_limit():
    """64 uneven small instances in one launch per kernel (graph replay): each
    equals the same instance run alone; a 65th is refused."""
    nhdc = _nhdc()
    rng = np.random.default_rng([2, 99])
    shapes = [(int(rng.integers(0, 2)), int(rng.integers(2, 13))) for _ in range(nhdc.MAX_INST)]
    cases = [_case(k, n, tag=i) for i, (k, n) in enumerate(shapes)]
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    b.step([c.dt for c in cases], 5, nsteps=2)
    for i, (c, d) in enumerate(zip(cases, ds)):
        alone, _ = _gpu(c, 2)
        _same(d.get_state(), alone, f"instance {i} R2B{shapes[i][0]}x{shapes[i][1]}")
    b.close()
    extra = nhdc.Dycore(cases[0])
    with pytest.raises(nhdc.NhdcError) as ei:
        nhdc.Batch(ds + [extra])
    assert ei.value.code == -1
    for d in ds + [extra]:
        d.close()


def test_full_size_r2b7_mixed_properties():
    """The R2B7x90 benchmark workload in the FP32-mixed form: one step stays
    finite and conserves dry mass and rho*theta_v to FP64 round-off (the
    oracle does not run at this size)."""
    c = CS.config_case(3)
    d = _nhdc().Dycore(c, precision="mixed")
    m0, r0 = d.diag()
    d.step(c.dt, c.nsub)
    d.check_finite()
    m1, r1 = d.diag()
    d.close()
    print(f"R2B7x90 mixed: mass {m1 / m0 - 1:.2e}  rho*theta_v {r1 / r0 - 1:.2e}", flush=True)
    assert abs(m1 / m0 - 1) <= 1e-13 and abs(r1 / r0 - 1) <= 1e-13


def test_full_size_r2b8_fp64_properties():
    """The R2B8x90 benchmark workload (the paper's 10 km grid, 5.24 M cells)
    in FP64, in the launch configuration the benchmark times (the starting
    shapes): one step stays finite and conserves dry mass and rho*theta_v to
    1e-13 relative; the same step from the same state with the level-parallel
    column and level tiles of 16 on every marching kind (other kernels, other
    block maps) gives the same state and mass fluxes to the bit.  The oracle
    does not run at this size."""
    print("R2B8x90: building the case", flush=True)
    c = CS.config_case(5)
    d = _nhdc().Dycore(c)
    start = d.shapes_in_use
    print("R2B8x90: starting shapes", start, flush=True)
    assert start[:3] == (0, 0, 0) and start[6] == 0
    m0, r0 = d.diag()
    d.step(c.dt, c.nsub)
    d.check_finite()
    m1, r1 = d.diag()
    a, fa = d.get_state(), d.mass_flux()
    print(f"R2B8x90 fp64: mass {m1 / m0 - 1:.2e}  rho*theta_v {r1 / r0 - 1:.2e}", flush=True)
    d.init_state(c.vn, c.w, c.rho, c.pi, c.theta_v)
    d.set_column_mode(1)
    d.set_tiles(16, 16, 16)
    print("R2B8x90: the same step, level-parallel column, tiles of 16", flush=True)
    d.step(c.dt, c.nsub)
    b, fb = d.get_state(), d.mass_flux()
    d.close()
    assert abs(m1 / m0 - 1) <= 1e-13 and abs(r1 / r0 - 1) <= 1e-13
    _same(a, b, "R2B8x90 two builds")
    assert np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])


def test_full_size_r2b6_all_options_one_step_bitwise():
    """The R2B6x90 benchmark workload with every option on (upwind edge
    values, fourth-order divergence damping, the w sponge, the diffusion of
    vn, four tracers), one step in the benchmark's launch configuration,
    against the oracle entry by entry."""
    c = CS.with_tracers(CS.with_params(CS.with_damping(CS.config_case(2)), upwind=1))
    d = _nhdc().Dycore(c)
    d.step(c.dt, c.nsub)
    gs, gq, gf = d.get_state(), d.get_tracers(), d.mass_flux()
    d.close()
    m = oracle.Model(c)
    m.step(c.dt, c.nsub)
    _same(gs, m.state(), "R2B6x90 all options")
    bad_q = int(np.count_nonzero(gq != m.tracers()))
    print("tracers differing entries", bad_q, flush=True)
    assert bad_q == 0
    of = m.flux()
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])
    assert np.all(gq[0] == 1.0)


def test_config2_recipe_ninety_levels_ten_steps_bitwise():
    """The benchmark's vertical grid (90 levels stretched to 75 km, terrain)
    on R2B4, ten steps against the oracle entry by entry."""
    c = CS.config_case(2, k=4)
    gs, gf = _gpu(c, 10)
    os_, of = _oracle(c, 10)
    _same(gs, os_, "R2B4x90 10 steps")
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_hundred_steps_conserve(precision):
    """R2B6x90, the benchmark's 100 steps: dry mass and sum rho theta_v
    conserved to 1e-13 relative (fixed-order device sums), state finite."""
    c = CS.config_case(2)
    d = _nhdc().Dycore(c, precision=precision)
    m0, r0 = d.diag()
    for _ in range(100):
        d.step(c.dt, c.nsub)
    d.check_finite()
    m1, r1 = d.diag()
    d.close()
    print(f"{precision} 100 steps: mass {m1 / m0 - 1:.2e}  rho*theta_v {r1 / r0 - 1:.2e}", flush=True)
    assert abs(m1 / m0 - 1) <= 1e-13 and abs(r1 / r0 - 1) <= 1e-13

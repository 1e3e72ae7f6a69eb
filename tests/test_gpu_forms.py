"""The other forms of the path through the C-ABI: level tiles and autotuning
(result-neutral), batching of uneven instances in one launch per kernel with
graph replay (bitwise equal to each instance alone, and so to the oracle in
FP64), and the FP32-mixed form (per-field error against FP64 next to the
FP32-rounding floor; FP64 mass fluxes keep mass conserved)."""
import os

import numpy as np
import pytest

import oracle
from paper_2511_02021_amd.inputs import case as CS

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def _run(case, steps, precision="fp64", tiles=None, state=None):
    d = _nhdc().Dycore(case, precision=precision)
    if state is not None:
        d.init_state(*[state[f] for f in ("vn", "w", "rho", "pi", "theta_v")])
    if tiles:
        d.set_tiles(*tiles)
    for _ in range(steps):
        d.step(case.dt, case.nsub)
    s = d.get_state()
    f = d.mass_flux()
    m = d.diag()
    d.close()
    return s, f, m


def test_level_tiles_are_result_neutral():
    c = CS.config_case(2, k=4, n_lev=30)
    ref, rf, _ = _run(c, 3)
    for tiles in ((16, 0, 0), (0, 8, 0), (0, 0, 16), (8, 8, 8), (7, 13, 5)):
        s, f, _ = _run(c, 3, tiles=tiles)
        for fld in FIELDS:
            assert np.array_equal(s[fld], ref[fld]), (tiles, fld)
        assert np.array_equal(f[0], rf[0]) and np.array_equal(f[1], rf[1])


def _batch_cases():
    return [CS.make_case(3, 20, z_top=30000.0, noise_seed=[0, 4, 0], dt=300.0),
            CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 4, 1],
                         noise_seed=[0, 4, 1], dt=150.0),
            CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 4, 2],
                         noise_seed=[0, 4, 2], dt=300.0)]


@pytest.mark.parametrize("tiles", [None, (16, 8, 16)])
def test_batch_equals_each_instance_and_oracle(tiles):
    nhdc = _nhdc()
    cases = _batch_cases()
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    if tiles:
        b.set_tiles(*tiles)
    b.step([c.dt for c in cases], 5, nsteps=3)
    for c, d in zip(cases, ds):
        s = d.get_state()
        m = oracle.Model(c)
        for _ in range(3):
            m.step(c.dt, 5)
        o = m.state()
        for f in FIELDS:
            assert np.array_equal(s[f], o[f]), (c.grid.k, c.n_lev, f)
    b.close()
    for d in ds:
        d.close()


def test_batch_graph_replay_after_changes():
    """Replays of the captured step, a change of dt (new capture) and a second
    batch over the same instances keep the bitwise agreement."""
    nhdc = _nhdc()
    cases = _batch_cases()
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    dts = [c.dt for c in cases]
    b.step(dts, 5, nsteps=2)
    b.step([x / 2 for x in dts], 5, nsteps=1)
    b.step(dts, 5, nsteps=1)
    b.close()
    b2 = nhdc.Batch(ds[:2])
    b2.step(dts[:2], 5, nsteps=1)
    b2.close()
    for i, (c, d) in enumerate(zip(cases, ds)):
        m = oracle.Model(c)
        seq = [c.dt, c.dt, c.dt / 2, c.dt] + ([c.dt] if i < 2 else [])
        for dt in seq:
            m.step(dt, 5)
        o, s = m.state(), d.get_state()
        for f in FIELDS:
            assert np.array_equal(s[f], o[f]), (i, f)
    for d in ds:
        d.close()


def test_batch_argument_errors():
    nhdc = _nhdc()
    c = CS.config_case(1, k=2)
    d = nhdc.Dycore(c)
    with pytest.raises(nhdc.NhdcError):
        nhdc.Batch([d, d])                      # same instance twice
    dm = nhdc.Dycore(c, precision="mixed")
    with pytest.raises(nhdc.NhdcError):
        nhdc.Batch([d, dm])                     # mixed precisions
    b = nhdc.Batch([d])
    with pytest.raises(nhdc.NhdcError) as ei:
        b.step([-1.0], 5)
    assert ei.value.code == -1
    b.close()
    d.close()
    dm.close()


def test_autotune_restores_state_and_caches(tmp_path):
    nhdc = _nhdc()
    c = CS.config_case(2, k=4, n_lev=30)
    d = nhdc.Dycore(c)
    d.step(c.dt, 5)
    before = d.get_state()
    path = str(tmp_path / "tune.json")
    best = d.autotune(c.dt, 5, cache_path=path)
    after = d.get_state()
    for f in FIELDS:
        assert np.array_equal(before[f], after[f]), f
    assert all(t in (0, 48, 32, 16, 8, 4) for t in best[:3]) and best[6] > 0
    assert best[3] in (64, 128, 256) and best[4] in (64, 128, 256) and best[5] in (0, 2, 3)
    assert len(best) == 8 and best[7] in (0, 1)  # the column mode
    txt = open(path).read()
    assert "fp64|launches|" in txt and str(c.grid.n_cells) in txt
    again = d.autotune(c.dt, 5, cache_path=path)   # cache hit: same shapes, no search
    assert again[:6] == best[:6] and abs(again[6] - best[6]) < 1e-5 and again[7] == best[7]
    d.step(c.dt, 5)
    ref, _, _ = _run(c, 2)
    s = d.get_state()
    for f in FIELDS:
        assert np.array_equal(s[f], ref[f]), f
    d.close()


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def mixed_error_table(case, steps, seed=7, precision="mixed"):
    """E_f: rel-L2 of (mixed - FP64) per field; S_f: the same norm between two
    FP64 runs whose initial states differ by seeded relative noise 2^-24.
    Both normalised by ||FP64|| and by ||FP64 - initial|| (the signal)."""
    init = dict(vn=case.vn, w=case.w, rho=case.rho, pi=case.pi, theta_v=case.theta_v)
    f64, _, _ = _run(case, steps)
    mix, _, mm = _run(case, steps, precision=precision)
    rng = np.random.default_rng(seed)
    pert = {k: v * (1.0 + 2.0 ** -24 * rng.standard_normal(v.shape)) for k, v in init.items()}
    f64p, _, _ = _run(case, steps, state=pert)
    table = {}
    for f in ("vn", "w", "rho", "pi", "theta_v"):
        signal = f64[f] - init[f]
        table[f] = dict(
            E=_rel_l2(mix[f], f64[f]), S=_rel_l2(f64p[f], f64[f]),
            E_signal=float(np.linalg.norm(mix[f] - f64[f]) / max(np.linalg.norm(signal), 1e-300)),
            S_signal=float(np.linalg.norm(f64p[f] - f64[f]) / max(np.linalg.norm(signal), 1e-300)))
    return table, mix


def test_mixed_form_error_and_conservation():
    c = CS.config_case(3, k=4, n_lev=30)   # the mixed-form recipe (terrain, 90-level stretch scaled)
    table, _ = mixed_error_table(c, 10)
    for f, r in table.items():
        print(f"mixed {f}: E={r['E']:.2e} S={r['S']:.2e} E/signal={r['E_signal']:.2e} "
              f"S/signal={r['S_signal']:.2e}", flush=True)
    for f, r in table.items():
        # the mixed form's deviation from FP64 stays below the FP32-rounding
        # floor of the same fields
        assert r["E"] <= r["S"], (f, r)
        assert r["E_signal"] < 1e-5, (f, r)
    # mass and rho*theta_v stay conserved to FP64 round-off (fluxes are FP64)
    d = _nhdc().Dycore(c, precision="mixed")
    m0, r0 = d.diag()
    for _ in range(10):
        d.step(c.dt, 5)
    m1, r1 = d.diag()
    d.close()
    assert abs(m1 / m0 - 1) <= 1e-13 and abs(r1 / r0 - 1) <= 1e-13


def test_mixed_batch_equals_mixed_alone():
    nhdc = _nhdc()
    cases = _batch_cases()
    alone = []
    for c in cases:
        s, _, _ = _run(c, 2, precision="mixed")
        alone.append(s)
    ds = [nhdc.Dycore(c, precision="mixed") for c in cases]
    b = nhdc.Batch(ds)
    b.step([c.dt for c in cases], 5, nsteps=2)
    for d, ref in zip(ds, alone):
        s = d.get_state()
        for f in FIELDS:
            assert np.array_equal(s[f], ref[f]), f
    b.close()
    for d in ds:
        d.close()


@pytest.mark.parametrize("option", ["upwind", "damped"])
def test_mixed_form_error_with_options(option):
    """The mixed form's per-field deviation from FP64 stays below the
    FP32-rounding floor with the upwind edge values and with the damping and
    diffusion options on."""
    c = CS.config_case(3, k=4, n_lev=30)
    c = CS.with_params(c, upwind=1) if option == "upwind" else CS.with_damping(c)
    table, _ = mixed_error_table(c, 10)
    for f, r in table.items():
        print(f"mixed {option} {f}: E={r['E']:.2e} S={r['S']:.2e} E/signal={r['E_signal']:.2e}",
              flush=True)
        assert r["E"] <= r["S"], (f, r)
        assert r["E_signal"] < 1e-5, (f, r)


def test_vn32_variant_error_and_conservation():
    """The mixed form with vn stored in FP32: its per-field deviation from FP64
    next to the FP32-rounding floor (reported; bar 10 S), mass and
    rho*theta_v conserved to FP64 round-off, vn at FP32 resolution."""
    c = CS.config_case(3, k=4, n_lev=30)
    table, mix = mixed_error_table(c, 10, precision="mixed_vn32")
    for f, r in table.items():
        print(f"mixed_vn32 {f}: E={r['E']:.2e} S={r['S']:.2e} E/signal={r['E_signal']:.2e}",
              flush=True)
        assert r["E"] <= 10 * r["S"], (f, r)
    # the stored vn is an FP32 number (the boundary returns it as FP64)
    assert np.array_equal(mix["vn"], mix["vn"].astype(np.float32).astype(np.float64))
    d = _nhdc().Dycore(c, precision="mixed_vn32")
    m0, r0 = d.diag()
    for _ in range(10):
        d.step(c.dt, 5)
    m1, r1 = d.diag()
    d.check_finite()
    d.close()
    assert abs(m1 / m0 - 1) <= 1e-13 and abs(r1 / r0 - 1) <= 1e-13


def test_vn32_batch_and_persistent_equal_alone():
    nhdc = _nhdc()
    cases = _batch_cases()
    alone = [_run(c, 2, precision="mixed_vn32")[0] for c in cases]
    for persistent in (False, True):
        ds = [nhdc.Dycore(c, precision="mixed_vn32") for c in cases]
        b = nhdc.Batch(ds)
        if persistent:
            b.set_persistent(True)
        b.step([c.dt for c in cases], 5, nsteps=2)
        for d, ref in zip(ds, alone):
            s = d.get_state()
            for f in FIELDS:
                assert np.array_equal(s[f], ref[f]), (persistent, f)
        b.close()
        for d in ds:
            d.close()

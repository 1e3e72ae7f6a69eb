"""Damping and diffusion around the substep on the HIP path, through the
C-ABI: fourth-order divergence damping, the Rayleigh sponge on w and the
Smagorinsky diffusion of vn, together and one at a time, in the FP64 form
bit for bit against the oracle with the same options; instances with and
without them in one batch; the mixed form's conservation with them; bad
option values refused."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2511_02021_amd.inputs import case as CS

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")
OFF = dict(div_damp4=0.0, smag=0.0, sponge_rate=0.0)


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def _gpu(case, steps, precision="fp64"):
    d = _nhdc().Dycore(case, precision=precision)
    for _ in range(steps):
        d.step(case.dt, case.nsub)
    s, f = d.get_state(), d.mass_flux()
    d.close()
    return s, f


def _oracle(case, steps):
    m = oracle.Model(case)
    for _ in range(steps):
        m.step(case.dt, case.nsub)
    return m.state(), m.flux()


def _same(a, b, label):
    bad = {f: int(np.count_nonzero(a[f] != b[f])) for f in FIELDS}
    print(label, "differing entries", bad, flush=True)
    assert not any(bad.values()), (label, bad)


def _flat():
    return CS.with_damping(CS.config_case(1), sponge_base=15000.0)


def _terrain(k=4, n_lev=30):
    return CS.with_damping(CS.config_case(2, k=k, n_lev=n_lev))


@pytest.mark.parametrize("which", ["flat R2B4x20", "terrain R2B4x30"])
def test_damped_fp64_matches_oracle_bitwise(which):
    c = _flat() if which.startswith("flat") else _terrain()
    gs, gf = _gpu(c, 10)
    os_, of = _oracle(c, 10)
    _same(gs, os_, f"damped {which} 10 steps")
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])


@pytest.mark.parametrize("option", ["div_damp4", "sponge", "smag"])
def test_each_option_alone_bitwise(option):
    base = CS.config_case(2, k=3, n_lev=20)
    kw = dict(OFF)
    kw.update({"div_damp4": dict(div_damp4=0.0025), "sponge": dict(sponge_rate=0.05),
               "smag": dict(smag=0.15)}[option])
    c = CS.with_damping(base, **kw)
    gs, gf = _gpu(c, 4)
    os_, of = _oracle(c, 4)
    _same(gs, os_, f"{option} alone")
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])
    plain, _ = _gpu(base, 4)
    assert not np.array_equal(plain["vn"], gs["vn"])


def test_damped_with_upwind_and_small_grids_bitwise():
    """The options combined with the upwind fluxes, and on the smallest
    ragged grids (a sponge over the top of two levels)."""
    up = _terrain(k=3, n_lev=24)
    up = dataclasses.replace(up, params=dataclasses.replace(up.params, upwind=1))
    for c, label in ((up, "upwind R2B3x24"),
                     (CS.with_damping(CS.make_case(0, 2, z_top=30000.0, terrain_seed=[9, 0],
                                                   noise_seed=[8, 0], dt=300.0),
                                      sponge_base=10000.0), "R2B0x2"),
                     (CS.with_damping(CS.make_case(1, 3, z_top=30000.0, terrain_seed=[9, 1],
                                                   noise_seed=[8, 1], dt=150.0),
                                      sponge_base=10000.0), "R2B1x3")):
        gs, _ = _gpu(c, 3)
        os_, _ = _oracle(c, 3)
        _same(gs, os_, label)


def test_damped_and_plain_instances_in_one_batch():
    nhdc = _nhdc()
    cases = [CS.make_case(3, 20, z_top=30000.0, noise_seed=[0, 8, 0], dt=300.0),
             CS.with_damping(CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 8, 1],
                                          noise_seed=[0, 8, 1], dt=150.0)),
             CS.with_damping(CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 8, 2],
                                          noise_seed=[0, 8, 2], dt=300.0), **{**OFF, "smag": 0.2})]
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    b.step([c.dt for c in cases], 5, nsteps=3)
    for i, (c, d) in enumerate(zip(cases, ds)):
        alone, _ = _gpu(c, 3)
        _same(d.get_state(), alone, f"instance {i}")
    b.close()
    for d in ds:
        d.close()


def test_damped_mixed_form_conserves_and_follows_fp64():
    c = _terrain()
    d = _nhdc().Dycore(c, precision="mixed")
    m0, r0 = d.diag()
    for _ in range(10):
        d.step(c.dt, c.nsub)
    d.check_finite()
    m1, r1 = d.diag()
    s = d.get_state()
    d.close()
    assert abs(m1 / m0 - 1) <= 1e-13 and abs(r1 / r0 - 1) <= 1e-13
    f64, _ = _gpu(c, 10)
    for f in ("vn", "rho", "theta_v"):
        rel = np.linalg.norm(s[f] - f64[f]) / np.linalg.norm(f64[f])
        print(f"damped mixed vs FP64 {f}: {rel:.2e}", flush=True)
        assert rel < 1e-5, f


def test_bad_option_values_are_refused():
    nhdc = _nhdc()
    base = CS.config_case(1, k=2)
    for kw in (dict(smag=-0.1), dict(div_damp4=float("nan"))):
        c = dataclasses.replace(base, params=dataclasses.replace(base.params, **kw))
        with pytest.raises(nhdc.NhdcError) as ei:
            nhdc.Dycore(c)
        assert ei.value.code == -1, kw
    wd = np.zeros(base.n_lev + 1)
    wd[3] = -1.0
    with pytest.raises(nhdc.NhdcError) as ei:
        nhdc.Dycore(dataclasses.replace(base, w_damp=wd))
    assert ei.value.code == -1

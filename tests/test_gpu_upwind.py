"""The second-order upwind option of the flux edge values on the HIP path,
through the C-ABI: the FP64 form against the oracle with the same option, bit
for bit; upwind and centred instances mixed in one batch, each equal to the
instance run alone; the FP32-mixed form's conservation with the option."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2511_02021_amd.inputs import case as CS

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def _upwind(case):
    return dataclasses.replace(case, params=dataclasses.replace(case.params, upwind=1))


def _gpu(case, steps, precision="fp64"):
    d = _nhdc().Dycore(case, precision=precision)
    for _ in range(steps):
        d.step(case.dt, case.nsub)
    s, f = d.get_state(), d.mass_flux()
    d.close()
    return s, f


def _same(a, b, label):
    bad = {f: int(np.count_nonzero(a[f] != b[f])) for f in FIELDS}
    print(label, "differing entries", bad, flush=True)
    assert not any(bad.values()), (label, bad)


@pytest.mark.parametrize("which", ["flat R2B4x20", "terrain R2B4x30"])
def test_upwind_fp64_matches_oracle_bitwise(which):
    base = CS.config_case(1) if which.startswith("flat") else CS.config_case(2, k=4, n_lev=30)
    c = _upwind(base)
    gs, gf = _gpu(c, 10)
    m = oracle.Model(c)
    for _ in range(10):
        m.step(c.dt, c.nsub)
    _same(gs, m.state(), f"upwind {which} 10 steps")
    of = m.flux()
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])
    # the option changes the solution
    cs, _ = _gpu(base, 10)
    assert not np.array_equal(cs["rho"], gs["rho"])


def test_upwind_and_centred_instances_in_one_batch():
    nhdc = _nhdc()
    cases = [CS.make_case(3, 20, z_top=30000.0, noise_seed=[0, 7, 0], dt=300.0),
             _upwind(CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 1],
                                  noise_seed=[0, 7, 1], dt=150.0)),
             CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 7, 2],
                          noise_seed=[0, 7, 2], dt=300.0)]
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    b.step([c.dt for c in cases], 5, nsteps=3)
    for i, (c, d) in enumerate(zip(cases, ds)):
        alone, _ = _gpu(c, 3)
        _same(d.get_state(), alone, f"instance {i} upwind={c.params.upwind}")
    b.close()
    for d in ds:
        d.close()


def test_upwind_mixed_form_conserves_mass():
    c = _upwind(CS.config_case(3, k=4, n_lev=30))
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
        print(f"upwind mixed vs FP64 {f}: {rel:.2e}", flush=True)
        assert rel < 1e-5, f

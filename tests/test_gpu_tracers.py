"""Tracer transport on the HIP path, through the C-ABI: FP64 bitwise
against the oracle (flat, terrain, with the upwind and damping options, the
smallest grids, one to four levels of PPM boundary handling), a constant
tracer kept to the bit in both forms, tracer mass conserved, a batch of
instances with and without tracers, and the argument checks."""
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


def _gpu(case, steps, precision="fp64"):
    d = _nhdc().Dycore(case, precision=precision)
    for _ in range(steps):
        d.step(case.dt, case.nsub)
    s, q = d.get_state(), d.get_tracers()
    d.close()
    return s, q


def _oracle(case, steps):
    m = oracle.Model(case)
    for _ in range(steps):
        m.step(case.dt, case.nsub)
    return m.state(), m.tracers()


def _same(gs, gq, os_, oq, label):
    bad = {f: int(np.count_nonzero(gs[f] != os_[f])) for f in FIELDS}
    bad["tracers"] = int(np.count_nonzero(gq != oq))
    print(label, "differing entries", bad, flush=True)
    assert gq.shape == oq.shape and not any(bad.values()), (label, bad)


def _small(k, n_lev):
    return CS.with_tracers(CS.make_case(k, n_lev, z_top=30000.0, terrain_seed=[9, k, n_lev],
                                        noise_seed=[8, k, n_lev], dt=300.0 / (k + 1)))


@pytest.mark.parametrize("which", ["flat R2B4x20", "terrain R2B4x30", "upwind+damped R2B3x30"])
def test_tracers_fp64_match_oracle_bitwise(which):
    if which.startswith("flat"):
        c = CS.with_tracers(CS.config_case(1))
    elif which.startswith("terrain"):
        c = CS.with_tracers(CS.config_case(2, k=4, n_lev=30))
    else:
        c = CS.with_damping(CS.config_case(2, k=3, n_lev=30))
        c = CS.with_tracers(CS.with_params(c, upwind=1))
    gs, gq = _gpu(c, 10)
    os_, oq = _oracle(c, 10)
    _same(gs, gq, os_, oq, which)
    assert np.all(gq[0] == 1.0)


@pytest.mark.parametrize("k,n_lev", [(0, 2), (1, 3), (2, 4), (2, 5), (1, 256)])
def test_tracers_small_grids_and_level_counts_bitwise(k, n_lev):
    """Two and three levels (linear interfaces only), four and five (the
    first interior cubic interfaces) and the library's maximum of 256."""
    c = _small(k, n_lev)
    gs, gq = _gpu(c, 3)
    os_, oq = _oracle(c, 3)
    _same(gs, gq, os_, oq, f"R2B{k}x{n_lev}")


def test_constant_tracer_and_tracer_mass_in_both_forms():
    c = CS.with_tracers(CS.config_case(2, k=5, n_lev=60))
    vol = c.grid.cell_area[None, :] * (c.zh[:-1] - c.zh[1:])
    for prec in ("fp64", "mixed"):
        d = _nhdc().Dycore(c, precision=prec)
        q0 = d.get_tracers()
        M0 = np.array([np.sum(vol * c.rho * q) for q in q0])
        for _ in range(5):
            d.step(c.dt, c.nsub)
        q, s = d.get_tracers(), d.get_state()
        d.close()
        M = np.array([np.sum(vol * s["rho"] * qt) for qt in q])
        print(prec, "tracer mass drift", np.abs(M / M0 - 1).max(), flush=True)
        assert np.all(q[0] == 1.0), prec
        assert np.abs(M / M0 - 1).max() <= 1e-12, prec
        assert np.all(np.isfinite(q)) and not np.array_equal(q[1], q0[1])


def test_tracer_and_plain_instances_in_one_batch():
    nhdc = _nhdc()
    cases = [CS.with_tracers(CS.make_case(3, 20, z_top=30000.0, noise_seed=[0, 9, 0], dt=300.0)),
             CS.make_case(4, 30, z_top=75000.0, stretch=1.6, terrain_seed=[1, 9, 1],
                          noise_seed=[0, 9, 1], dt=150.0),
             CS.with_tracers(CS.make_case(3, 45, z_top=75000.0, stretch=1.6, terrain_seed=[1, 9, 2],
                                          noise_seed=[0, 9, 2], dt=300.0), names=("h2o", "o3"))]
    ds = [nhdc.Dycore(c) for c in cases]
    b = nhdc.Batch(ds)
    with pytest.raises(nhdc.NhdcError) as ei:
        ds[0].set_tracers(cases[0].tracers)   # refused while batched
    assert ei.value.code == -5
    b.step([c.dt for c in cases], 5, nsteps=3)
    for i, (c, d) in enumerate(zip(cases, ds)):
        alone_s, alone_q = _gpu(c, 3)
        _same(d.get_state(), d.get_tracers(), alone_s, alone_q, f"instance {i}")
    b.close()
    for d in ds:
        d.close()


def test_tracer_argument_checks():
    nhdc = _nhdc()
    c = CS.config_case(1, k=2)
    d = nhdc.Dycore(c)
    with pytest.raises(nhdc.NhdcError) as ei:
        d.set_tracers(np.ones((17, c.n_lev, c.grid.n_cells)))
    assert ei.value.code == -1
    d.set_tracers(np.ones((2, c.n_lev, c.grid.n_cells)))
    assert d.get_tracers().shape == (2, c.n_lev, c.grid.n_cells)
    d.set_tracers(np.zeros((0, c.n_lev, c.grid.n_cells)))   # removed
    assert d.get_tracers().shape[0] == 0
    d.step(c.dt, c.nsub)
    d.close()

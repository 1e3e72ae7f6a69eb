"""Plain FP64 HIP path against the FP64 CPU oracle, element by element, through
the C-ABI.  Bar: max |gpu - oracle| / max |oracle| <= 1e-12 per field after
10 steps; the FP64 kernels are in fact bitwise equal to the oracle (same
operations in the same order, no contraction), which one test asserts."""
import numpy as np
import pytest

import oracle
from paper_2511_02021_amd.inputs import case as CS
from paper_2511_02021_amd.inputs import grid as G

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _compare(gs, os_, tol, label):
    errs = {f: rel(gs[f], os_[f]) for f in FIELDS}
    print(label, {f: f"{e:.2e}" for f, e in errs.items()}, flush=True)
    for f, e in errs.items():
        assert e <= tol, (label, f, e)
    return errs


def _run_both(case, steps, dt=None, nsub=None):
    dt = case.dt if dt is None else dt
    nsub = case.nsub if nsub is None else nsub
    d = _nhdc().Dycore(case)
    m = oracle.Model(case)
    for _ in range(steps):
        d.step(dt, nsub)
        m.step(dt, nsub)
    gs = d.get_state()
    gf = d.mass_flux()
    d.close()
    return gs, gf, m.state(), m.flux()


@pytest.fixture(scope="module")
def cfg1():
    return CS.config_case(1)


def test_one_substep_matches_oracle(cfg1):
    gs, gf, os_, of = _run_both(cfg1, 1, dt=cfg1.dt / 5, nsub=1)
    _compare(gs, os_, 1e-13, "cfg1 1 substep")
    assert rel(gf[0], of[0]) <= 1e-13 and rel(gf[1], of[1]) <= 1e-13


def test_ten_steps_match_oracle_flat(cfg1):
    gs, gf, os_, of = _run_both(cfg1, 10)
    _compare(gs, os_, 1e-12, "cfg1 10 steps")
    assert rel(gf[0], of[0]) <= 1e-12 and rel(gf[1], of[1]) <= 1e-12


def test_ten_steps_match_oracle_terrain():
    c = CS.config_case(2, k=4, n_lev=30)   # terrain recipe, 30 stretched levels to 75 km
    gs, gf, os_, of = _run_both(c, 10)
    _compare(gs, os_, 1e-12, "R2B4x30 terrain 10 steps")
    assert rel(gf[0], of[0]) <= 1e-12 and rel(gf[1], of[1]) <= 1e-12


def test_fp64_form_is_bitwise_equal_to_oracle():
    """The FP64 kernels form every value with the oracle's operations in the
    oracle's order and without contraction: the results agree to the last bit."""
    c = CS.config_case(2, k=4, n_lev=30)
    gs, gf, os_, of = _run_both(c, 3)
    diff = {f: int(np.count_nonzero(gs[f] != os_[f])) for f in FIELDS}
    print("bitwise differing entries", diff, flush=True)
    assert all(v == 0 for v in diff.values()), diff
    assert np.array_equal(gf[0], of[0]) and np.array_equal(gf[1], of[1])


def test_full_size_r2b6_one_step():
    """The benchmark workload (R2B6, 90 levels to 75 km, terrain, dt 90 s, 5
    substeps), one full step in the launch configuration the benchmark times."""
    c = CS.config_case(2)
    gs, gf, os_, of = _run_both(c, 1)
    _compare(gs, os_, 1e-12, "R2B6x90 1 step")
    assert rel(gf[0], of[0]) <= 1e-12 and rel(gf[1], of[1]) <= 1e-12


def test_full_size_r2b6_ten_steps():
    """The R2B6x90 workload's grid for 10 steps (the oracle's part takes about
    a minute and a half on the host's threads): every field within 1e-12 of
    the oracle, and bitwise equal."""
    c = CS.config_case(2)
    print("R2B6x90, 10 steps on both sides", flush=True)
    gs, gf, os_, of = _run_both(c, 10)
    _compare(gs, os_, 1e-12, "R2B6x90 10 steps")
    assert rel(gf[0], of[0]) <= 1e-12 and rel(gf[1], of[1]) <= 1e-12
    diff = {f: int(np.count_nonzero(gs[f] != os_[f])) for f in FIELDS}
    print("bitwise differing entries", diff, flush=True)
    assert all(v == 0 for v in diff.values()), diff


def test_run_to_run_bitwise(cfg1):
    out = []
    for _ in range(2):
        d = _nhdc().Dycore(cfg1)
        for _ in range(3):
            d.step(cfg1.dt, 5)
        out.append(d.get_state())
        d.close()
    for f in FIELDS:
        assert np.array_equal(out[0][f], out[1][f]), f


def test_numbering_invariance_on_gpu():
    ref = None
    for order, seed in (("sfc", 0), ("random", 3)):
        canon, gr = G.build_grid(4, order=order, seed=seed, with_canonical=True)
        c = CS.config_case(2, k=4, n_lev=20, grids=(canon, gr))
        d = _nhdc().Dycore(c)
        d.step(c.dt, 5)
        s = d.get_state()
        d.close()
        ic, ie = np.argsort(gr.canon_cell), np.argsort(gr.canon_edge)
        back = {f: (v[:, ie] if f == "vn" else v[:, ic]) for f, v in s.items()}
        if ref is None:
            ref = back
        else:
            for f in FIELDS:
                assert np.array_equal(ref[f], back[f]), f


def test_rest_state_stays_at_rest_on_gpu():
    p = CS.Params(div_damp=0.0)
    c = CS.make_case(4, 20, z_top=30000.0, sigma=0.0, dt=300.0, params=p)
    d = _nhdc().Dycore(c)
    for _ in range(100):
        d.step(c.dt, 5)
    s = d.get_state()
    assert np.abs(s["vn"]).max() <= 1e-11 and np.abs(s["w"]).max() <= 1e-11
    for f in ("rho", "pi", "theta_v"):
        assert np.abs(s[f] / getattr(c, f) - 1).max() <= 1e-13, f


def test_mass_conserved_on_gpu():
    c = CS.config_case(2, k=5, n_lev=40)
    d = _nhdc().Dycore(c)
    m0, r0 = d.diag()
    m = oracle.Model(c)
    om0, or0 = m.diag()
    assert abs(m0 / om0 - 1) < 1e-13 and abs(r0 / or0 - 1) < 1e-13
    for _ in range(20):
        d.step(c.dt, 5)
    m1, r1 = d.diag()
    d.check_finite()
    assert abs(m1 / m0 - 1) <= 1e-13 and abs(r1 / r0 - 1) <= 1e-13


def test_argument_and_state_errors():
    nhdc = _nhdc()
    c = CS.config_case(1, k=2)
    d = nhdc.Dycore(c, init=False)
    with pytest.raises(nhdc.NhdcError) as ei:
        d.step(1.0, 1)
    assert ei.value.code == -5
    d.init_state(c.vn, c.w, c.rho, c.pi, c.theta_v)
    for dt, ns in ((0.0, 1), (-1.0, 1), (float("nan"), 1), (10.0, 0)):
        with pytest.raises(nhdc.NhdcError) as ei:
            d.step(dt, ns)
        assert ei.value.code == -1
    d.close()


def test_invalid_grid_rejected():
    nhdc = _nhdc()
    c = CS.config_case(1, k=2)
    bad = CS.replace(c, grid=CS.replace(c.grid, cell_edges=c.grid.cell_edges.copy()))
    bad.grid.cell_edges[1, 5] = bad.grid.n_edges + 3
    with pytest.raises(nhdc.NhdcError) as ei:
        nhdc.Dycore(bad)
    assert ei.value.code == -4
    zh = c.zh.copy()
    zh[3, 7] = zh[4, 7] - 1.0
    with pytest.raises(nhdc.NhdcError) as ei:
        nhdc.Dycore(CS.replace(c, zh=zh))
    assert ei.value.code == -4

"""Synthetic case generator: spherical-harmonic terrain against scipy, the
vertical coordinate, the reference profile against its defining ODE, the
discrete hydrostatic balance, the equation of state and the noise recipe."""
import numpy as np
import pytest
from scipy.special import sph_harm_y

from paper_2511_02021_amd.inputs import case as CS


def _unit_points(n, seed=0):
    x = np.random.default_rng(seed).standard_normal((3, n))
    return x / np.linalg.norm(x, axis=0)


@pytest.mark.parametrize("l,m", [(1, 0), (1, 1), (1, -1), (2, 2), (5, -3), (8, 0), (17, 11),
                                 (32, -32), (32, 5)])
def test_real_harmonics_match_scipy(l, m):
    lmax = 32
    xyz = _unit_points(400, seed=l * 100 + m)
    coef = np.zeros((lmax + 1) ** 2 - 1)
    coef[l * l - 1 + m + l] = 1.0
    got = CS.harmonic_sum(xyz, coef, lmax)
    theta = np.arccos(np.clip(xyz[2], -1, 1))
    phi = np.arctan2(xyz[1], xyz[0])
    y = sph_harm_y(l, abs(m), theta, phi)  # includes the Condon-Shortley phase
    cs = (-1.0) ** abs(m)
    if m == 0:
        ref = y.real
    elif m > 0:
        ref = np.sqrt(2.0) * cs * y.real
    else:
        ref = np.sqrt(2.0) * cs * y.imag
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


def test_terrain_range_and_seed():
    c = CS.config_case(2, k=3, n_lev=30)
    assert c.h.min() == 0.0 and abs(c.h.max() - 3000.0) < 1e-9
    c2 = CS.config_case(2, k=3, n_lev=30)
    assert np.array_equal(c.h, c2.h)
    c3 = CS.config_case(3, k=3, n_lev=30)
    assert not np.array_equal(c.h, c3.h)


def test_vertical_coordinate():
    c = CS.config_case(2, k=3, n_lev=90)
    zh = c.zh
    assert np.all(np.diff(zh, axis=0) < 0)                       # strictly decreasing downward
    assert np.allclose(zh[0], 75000.0) and np.array_equal(zh[-1], c.h)
    flat = CS.flat_coordinate(90, 75000.0, 1.6)
    assert 50 < flat[-2] < 60 and 1300 < flat[0] - flat[1] < 1360  # ~56 m bottom, ~1.33 km top
    above = flat >= CS.Z_FLAT
    assert np.array_equal(zh[above], np.broadcast_to(flat[above, None], zh[above].shape))
    # thickest terrain: lowest layer keeps >= 0.6 of its flat thickness
    dz = zh[-2] - zh[-1]
    assert dz.min() >= 0.6 * (flat[-2] - flat[-1])


def test_reference_profile_solves_hydrostatic_ode():
    c = CS.config_case(2, k=2, n_lev=90)
    z = 0.5 * (c.zh[:-1] + c.zh[1:])
    p = c.params
    tref = CS.T_REF_TOP + CS.T_REF_DELTA * np.exp(-z / CS.T_REF_SCALE)
    assert np.allclose(c.theta_ref * c.pi_ref, tref, rtol=1e-14, atol=0)
    # d(ln pi)/dz = -g/(cpd T_ref), checked by a centred difference of the closed form
    zz = np.linspace(10.0, 74000.0, 200)
    f = lambda zq: -p.grav / (p.cpd * CS.T_REF_TOP) * (
        zq + CS.T_REF_SCALE * np.log((CS.T_REF_TOP + CS.T_REF_DELTA * np.exp(-zq / CS.T_REF_SCALE)) /
                                     (CS.T_REF_TOP + CS.T_REF_DELTA)))
    hdz = 1e-2
    dln = (f(zz + hdz) - f(zz - hdz)) / (2 * hdz)
    ode = -p.grav / (p.cpd * (CS.T_REF_TOP + CS.T_REF_DELTA * np.exp(-zz / CS.T_REF_SCALE)))
    assert np.allclose(dln, ode, rtol=1e-8)


@pytest.mark.parametrize("terrain", [False, True])
def test_discrete_hydrostatic_balance(terrain):
    c = CS.config_case(2, k=3, n_lev=60) if terrain else CS.config_case(1, k=3)
    p = c.params
    zh, pr, tr, pi, th = c.zh, c.pi_ref, c.theta_ref, c.pi, c.theta_v
    z = 0.5 * (zh[:-1] + zh[1:])
    g = (z[:-1] - zh[1:-1]) / (z[:-1] - z[1:])
    dzh = z[:-1] - z[1:]
    interp = lambda f: g * f[1:] + (1 - g) * f[:-1]
    dref = -p.grav / (p.cpd * interp(tr))
    pp = pi - pr
    t1 = interp(th) * (pp[:-1] - pp[1:]) / dzh
    t2 = interp(th - tr) * dref
    # residual at the round-off floor: Exner values carry a relative error of one
    # unit roundoff, so the difference quotient carries u*theta*(|pi_a|+|pi_b|)/dzh
    u = np.finfo(float).eps / 2
    floor = u * (interp(th) * (np.abs(pi[:-1]) + np.abs(pi[1:])) / dzh + np.abs(t2))
    assert np.all(np.abs(t1 + t2) <= 8 * floor)
    # isothermal: theta_v * pi = T0; ideal gas p = rho Rd T with p = p00 pi^(cpd/Rd)
    assert np.allclose(th * pi, CS.T0, rtol=1e-15, atol=0)
    pres = p.p00 * pi ** (p.cpd / p.rd)
    assert np.allclose(pres, c.rho * p.rd * CS.T0, rtol=1e-13, atol=0)
    # bottom level starts from the analytic isothermal value
    assert np.allclose(pi[-1], np.exp(-p.grav * z[-1] / (p.cpd * CS.T0)), rtol=1e-15)


def test_noise_recipe():
    c = CS.config_case(1, k=3)
    rms = np.sqrt((c.vn ** 2).mean(axis=1))
    assert np.allclose(rms, 1.0, rtol=1e-12)
    assert np.all(c.w == 0)
    # levels independent, seeded
    assert abs(np.corrcoef(c.vn[0], c.vn[1])[0, 1]) < 0.1
    c2 = CS.config_case(1, k=3)
    assert np.array_equal(c.vn, c2.vn)
    # smoothing: neighbouring edges correlate strongly after three passes
    g = c.grid
    e0, e1 = g.cell_edges[0], g.cell_edges[1]
    raw = np.random.default_rng([0, 1, 0]).standard_normal((20, g.n_edges))[:, g.canon_edge]
    corr = lambda x: np.abs(np.corrcoef(np.abs(x[0, e0]), np.abs(x[0, e1]))[0, 1])
    assert corr(c.vn) > corr(raw) + 0.1


def test_case_is_numbering_independent():
    a = CS.config_case(2, k=3, n_lev=30, order="canonical")
    b = CS.config_case(2, k=3, n_lev=30, order="sfc")
    ic, ie = b.grid.canon_cell, b.grid.canon_edge
    for f in ("zh", "pi_ref", "theta_ref", "rho", "pi", "theta_v", "w"):
        assert np.array_equal(getattr(a, f)[:, ic], getattr(b, f)), f
    assert np.array_equal(a.vn[:, ie], b.vn)


def test_batch_shapes_recipe():
    shapes = CS.batch_shapes()
    assert len(shapes) == 16
    assert all(k in (4, 5, 6) and 30 <= n <= 90 for k, n in shapes)
    assert shapes == CS.batch_shapes()

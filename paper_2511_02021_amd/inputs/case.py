"""Seeded synthetic cases for the dynamical-core substep.

The paper initialises its km-scale run from reanalysis over real topography
(Sec. 4.1) on the grids of Table 2 with 90 levels; neither data set exists
here, so every case is generated from a recipe with the same shapes:

* vertical grid: N full levels between a flat coordinate zeta (linear to
  30 km, or zeta = z_top * x**1.6 to 75 km) and terrain-following heights
  z = zeta + h * b(zeta), b a sinh decay that is 0 above 16 km (scale 8 km);
* terrain: random real spherical harmonics of degree 1..32 with coefficients
  N(0, (l+1)**-2) drawn from ``default_rng([1, cfg, inst])``, min-max scaled
  to [0, 3000] m;
* reference profile T_ref(z) = 213.15 K + 75 K * exp(-z / 10 km) with its
  exact hydrostatic Exner function;
* initial state: dry isothermal 250 K atmosphere in discrete hydrostatic
  balance of the resting w-equation, plus normal-velocity noise (standard
  normals from ``default_rng([0, cfg, inst])``, smoothed by three sign-aware
  passes, unit RMS per level, times sigma = 1 m/s).

Everything is generated in canonical numbering, then permuted to the grid's
numbering, so one recipe gives the same physical state in every numbering.
"""
import ctypes as C
from dataclasses import dataclass, field, replace

import numpy as np

from . import grid as G


@dataclass(frozen=True)
class Params:
    """Physical constants and scheme coefficients of the substep."""
    radius: float = G.EARTH_RADIUS
    omega: float = 7.29212e-5       # planetary rotation [1/s]
    grav: float = 9.80665
    rd: float = 287.04
    cpd: float = 1004.64
    p00: float = 1.0e5
    beta: float = 0.65              # implicit weight of the vertical solve
    wgt_corr: float = 0.75          # weight of the corrector tendency
    extrap: float = 1.0 / 3.0       # Exner extrapolation factor
    div_damp: float = 0.01          # second-order divergence damping coefficient
    upwind: int = 0                 # edge rho, theta_v in fluxes: 0 centred, 1 second-order upwind
    div_damp4: float = 0.0          # fourth-order divergence damping coefficient (0: off)
    smag: float = 0.0               # Smagorinsky constant of the diffusion of vn (0: off)

    @property
    def cvd(self):
        return self.cpd - self.rd


# background and reference profile of every case
T0 = 250.0
T_REF_TOP, T_REF_DELTA, T_REF_SCALE = 213.15, 75.0, 10000.0
Z_FLAT, DECAY_SCALE = 16000.0, 8000.0
H_MAX, L_MAX = 3000.0, 32


@dataclass
class Case:
    grid: G.Grid
    n_lev: int
    params: Params
    dt: float
    nsub: int
    zh: np.ndarray          # [N+1, nc] half-level heights, top to bottom
    pi_ref: np.ndarray      # [N, nc]
    theta_ref: np.ndarray   # [N, nc]
    vn: np.ndarray          # [N, ne]
    w: np.ndarray           # [N+1, nc]
    rho: np.ndarray         # [N, nc]
    pi: np.ndarray          # [N, nc] Exner pressure
    theta_v: np.ndarray     # [N, nc]
    h: np.ndarray           # [nc] surface height
    zeta: np.ndarray = None  # [N+1] flat coordinate of the half levels
    w_damp: np.ndarray = None  # [N+1] Rayleigh damping rate of w per half level [1/s], or None
    tracers: np.ndarray = None  # [nt, N, nc] tracer mixing ratios, or None
    meta: dict = field(default_factory=dict)

    @property
    def state(self):
        return dict(vn=self.vn, w=self.w, rho=self.rho, pi=self.pi, theta_v=self.theta_v)

    @property
    def cell_levels(self):
        return self.grid.n_cells * self.n_lev


def _lib():
    lib = G.lib()
    if not hasattr(lib, "_case_ready"):
        lib.nhcase_terrain.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p]
        lib.nhcase_columns.argtypes = [C.c_void_p] + [C.c_void_p] * 6
        lib.nhcase_smooth_noise.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        lib._case_ready = True
    return lib


class _ColumnArgs(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_lev", C.c_int32), ("balanced", C.c_int32),
                ("zeta", C.c_void_p), ("h", C.c_void_p), ("z_flat", C.c_double),
                ("decay_scale", C.c_double), ("grav", C.c_double), ("cpd", C.c_double),
                ("rd", C.c_double), ("p00", C.c_double), ("t0", C.c_double),
                ("t_ref_top", C.c_double), ("t_ref_delta", C.c_double),
                ("t_ref_scale", C.c_double)]


class _GridArgs(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_edges", C.c_int64), ("radius", C.c_double)] + [
        (n, C.c_void_p) for n in ("cell_edges", "cell_sign", "edge_cells", "cell_x", "cell_area",
                                  "edge_x", "edge_normal", "edge_length")]


def _ptr(a):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def flat_coordinate(n_lev, z_top, stretch):
    """Half-level heights zeta_i, i = 1..N+1 (top to bottom) over flat ground."""
    x = (n_lev - np.arange(n_lev + 1, dtype=np.float64)) / n_lev
    return z_top * x if stretch == 1.0 else z_top * x ** stretch


def harmonic_sum(xyz, coef, lmax):
    """sum_{l=1..lmax} sum_{m=-l..l} coef[l*l-1+m+l] Y_lm(xyz) for unit vectors xyz [3, n]
    (real orthonormal harmonics without the Condon-Shortley phase)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    assert coef.size == (lmax + 1) ** 2 - 1
    out = np.empty(xyz.shape[1])
    rc = _lib().nhcase_terrain(_ptr(xyz), xyz.shape[1], int(lmax), _ptr(coef), _ptr(out))
    if rc != 0:
        raise RuntimeError("nhcase_terrain failed")
    return out


def terrain(grid_canon, seed):
    """Seeded random-harmonic terrain at cell centres, scaled to [0, H_MAX]."""
    rng = np.random.default_rng(seed)
    coef = np.concatenate([rng.normal(0.0, 1.0 / (l + 1.0), size=2 * l + 1)
                           for l in range(1, L_MAX + 1)])
    raw = harmonic_sum(grid_canon.cell_x, coef, L_MAX)
    return H_MAX * (raw - raw.min()) / (raw.max() - raw.min())


def columns(zeta, h, params, balanced=True):
    nc, n_lev = h.size, zeta.size - 1
    zh = np.empty((n_lev + 1, nc))
    out = [np.empty((n_lev, nc)) for _ in range(5)]
    a = _ColumnArgs(nc, n_lev, int(balanced), _ptr(zeta), _ptr(h), Z_FLAT, DECAY_SCALE,
                    params.grav, params.cpd, params.rd, params.p00, T0,
                    T_REF_TOP, T_REF_DELTA, T_REF_SCALE)
    rc = _lib().nhcase_columns(C.byref(a), _ptr(zh), *[_ptr(o) for o in out])
    if rc != 0:
        raise RuntimeError(f"nhcase_columns failed ({rc})")
    pi_ref, theta_ref, pi, theta_v, rho = out
    return zh, pi_ref, theta_ref, pi, theta_v, rho


def smoothed_noise(grid_canon, n_lev, seed, passes=3):
    x = np.random.default_rng(seed).standard_normal((n_lev, grid_canon.n_edges))
    g = grid_canon
    a = _GridArgs(g.n_cells, g.n_edges, g.radius, _ptr(g.cell_edges), _ptr(g.cell_sign),
                  _ptr(g.edge_cells), _ptr(g.cell_x), _ptr(g.cell_area), _ptr(g.edge_x),
                  _ptr(g.edge_normal), _ptr(g.edge_length))
    rc = _lib().nhcase_smooth_noise(C.byref(a), n_lev, passes, _ptr(x))
    if rc != 0:
        raise RuntimeError("nhcase_smooth_noise failed")
    return x


def latitude(grid):
    return np.arcsin(np.clip(grid.cell_x[2], -1.0, 1.0))


def legendre(l, x):
    return np.polynomial.legendre.Legendre.basis(l)(x)


def make_case(k, n_lev, z_top=30000.0, stretch=1.0, terrain_seed=None, noise_seed=None,
              sigma=1.0, dt=300.0, nsub=5, order="curve", balanced=True, gravity_wave=None,
              params=Params(), grids=None, meta=None):
    """Build one case.  ``terrain_seed`` is a seed of the random terrain, a
    callable mapping the canonical grid to surface heights, or None (flat).
    ``gravity_wave`` = (epsilon, degree) adds the small
    potential-temperature bump e^{z/2H} sin(pi z/z_top) P_l(sin lat) at fixed
    Exner pressure.  ``grids`` may pass a prebuilt (canonical, renumbered) pair."""
    canon, g = grids if grids is not None else G.build_grid(k, order=order, with_canonical=True)
    nc = canon.n_cells
    if callable(terrain_seed):
        h = np.ascontiguousarray(terrain_seed(canon), dtype=np.float64)
    elif terrain_seed is not None:
        h = terrain(canon, terrain_seed)
    else:
        h = np.zeros(nc)
    zeta = flat_coordinate(n_lev, z_top, stretch)
    zh, pi_ref, theta_ref, pi, theta_v, rho = columns(zeta, h, params, balanced)
    if gravity_wave is not None:
        eps, deg = gravity_wave
        z = 0.5 * (zh[:-1] + zh[1:])
        H = params.rd * T0 / params.grav
        bump = eps * np.exp(z / (2 * H)) * np.sin(np.pi * z / z_top) * legendre(
            deg, np.sin(latitude(canon)))[None, :]
        theta_v = theta_v * (1.0 + bump)
        rho = params.p00 * pi ** (params.cvd / params.rd) / (params.rd * theta_v)
    if noise_seed is not None and sigma != 0.0:
        vn = sigma * smoothed_noise(canon, n_lev, noise_seed)
    else:
        vn = np.zeros((n_lev, canon.n_edges))
    w = np.zeros((n_lev + 1, nc))
    if g is not canon:
        zh, pi_ref, theta_ref, pi, theta_v, rho, w = G.permute_grid_fields(
            g, [zh, pi_ref, theta_ref, pi, theta_v, rho, w], "cell")
        (h,) = G.permute_grid_fields(g, [h], "cell")
        (vn,) = G.permute_grid_fields(g, [vn], "edge")
    return Case(grid=g, n_lev=n_lev, params=params, dt=dt, nsub=nsub, zh=zh, pi_ref=pi_ref,
                theta_ref=theta_ref, vn=vn, w=w, rho=rho, pi=pi, theta_v=theta_v, h=h,
                zeta=np.ascontiguousarray(zeta), meta=dict(meta or {}))


# Named workloads.  dt of R2B7/R2B8 keeps the horizontal sound Courant number
# of the R2B4/R2B6 cases; 5 substeps per step throughout.
CONFIGS = {
    1: dict(k=4, n_lev=20, z_top=30000.0, stretch=1.0, terrain=False, dt=300.0, steps=10,
            precision="fp64"),
    2: dict(k=6, n_lev=90, z_top=75000.0, stretch=1.6, terrain=True, dt=90.0, steps=100,
            precision="fp64"),
    3: dict(k=7, n_lev=90, z_top=75000.0, stretch=1.6, terrain=True, dt=45.0, steps=100,
            precision="mixed"),
    5: dict(k=8, n_lev=90, z_top=75000.0, stretch=1.6, terrain=True, dt=22.5, steps=50,
            precision="mixed"),
}
BATCH_DT = {4: 300.0, 5: 150.0, 6: 90.0}


def config_case(cfg, inst=0, order="curve", k=None, n_lev=None, **kw):
    """Case of a named workload; ``k``/``n_lev`` override the grid size
    (smaller stand-ins of the same recipe for tests)."""
    c = CONFIGS[cfg]
    return make_case(k if k is not None else c["k"], n_lev if n_lev is not None else c["n_lev"],
                     z_top=c["z_top"], stretch=c["stretch"],
                     terrain_seed=[1, cfg, inst] if c["terrain"] else None,
                     noise_seed=[0, cfg, inst], dt=c["dt"], nsub=5, order=order,
                     meta=dict(config=cfg, inst=inst), **kw)


def batch_shapes(n=16, seed=(2, 4, 0)):
    """(k_i, N_i) of the uneven batch: k uniform in {4,5,6}, N uniform in [30, 90]."""
    rng = np.random.default_rng(list(seed))
    ks = rng.integers(4, 7, size=n)
    ns = rng.integers(30, 91, size=n)
    return [(int(a), int(b)) for a, b in zip(ks, ns)]


def batch_cases(n=16, order="curve"):
    out = []
    for i, (k, nl) in enumerate(batch_shapes(n)):
        out.append(make_case(k, nl, z_top=75000.0, stretch=1.6, terrain_seed=[1, 4, i],
                             noise_seed=[0, 4, i], dt=BATCH_DT[k], nsub=5, order=order,
                             meta=dict(config=4, inst=i)))
    return out


def with_params(case, **kw):
    return replace(case, params=replace(case.params, **kw))


TRACER_NAMES = ("one", "h2o", "o3", "co2")


def tracer_set(case, names=TRACER_NAMES):
    """Synthetic tracer mixing ratios [nt, N, nc] with the vertical and
    meridional shapes of the paper's tracers (H2O, O3, CO2), plus a constant
    one: water vapour decaying with height (scale 2.5 km, moist tropics),
    ozone peaked near 25 km, carbon dioxide nearly uniform (1 % in P_3 of
    latitude); heights are the full-level heights of each column."""
    z = 0.5 * (case.zh[:-1] + case.zh[1:])
    s = np.sin(latitude(case.grid))[None, :]
    shapes = {
        "one": np.ones_like(z),
        "h2o": 0.015 * np.exp(-z / 2500.0) * (0.3 + 0.7 * (1.0 - s ** 2)),
        "o3": 8e-6 * np.exp(-((z - 25000.0) / 7000.0) ** 2) * (1.0 + 0.3 * s),
        "co2": 4.2e-4 * (1.0 + 0.01 * legendre(3, s)) * np.ones_like(z),
    }
    return np.ascontiguousarray(np.stack([shapes[n] for n in names]))


def with_tracers(case, names=TRACER_NAMES):
    return replace(case, tracers=tracer_set(case, names))


def sponge_profile(zeta, rate, z_base):
    """Rayleigh damping rate of w at the half levels of the flat coordinate
    zeta: Klemp's profile, rate * sin^2(pi/2 (zeta - z_base)/(z_top - z_base))
    above z_base, 0 below (z_top = zeta[0], the lid)."""
    zeta = np.asarray(zeta, dtype=np.float64)
    x = np.clip((zeta - z_base) / (zeta[0] - z_base), 0.0, 1.0)
    return np.ascontiguousarray(rate * np.sin(0.5 * np.pi * x) ** 2)


# damping and diffusion around the substep, all three on: fourth-order
# divergence damping, a sponge over the top third of a 75 km column (rate
# 0.05 /s at the lid), Smagorinsky diffusion of vn with c_s = 0.15
DAMPED = dict(div_damp4=0.0025, smag=0.15, sponge_rate=0.05, sponge_base=50000.0)


def with_damping(case, div_damp4=DAMPED["div_damp4"], smag=DAMPED["smag"],
                 sponge_rate=DAMPED["sponge_rate"], sponge_base=DAMPED["sponge_base"]):
    """The case with the damping and diffusion options set (a rate of 0 or a
    base at or above the lid leaves the sponge off)."""
    wd = None
    if sponge_rate > 0.0 and sponge_base < case.zeta[0]:
        wd = sponge_profile(case.zeta, sponge_rate, sponge_base)
    return replace(case, params=replace(case.params, div_damp4=div_damp4, smag=smag), w_damp=wd)

"""Seeded synthetic inputs of the dynamical core: the icosahedral grid with its
space-filling-curve renumbering (``grid``) and the case generator (``case``:
vertical grid, terrain, reference profile, balanced initial state, velocity
noise).  Nothing here computes a step of the method; both the CPU oracle and
the HIP library consume these arrays unchanged."""
from .grid import Grid, build_grid, grid_counts  # noqa: F401
from .case import Case, Params, make_case, CONFIGS  # noqa: F401

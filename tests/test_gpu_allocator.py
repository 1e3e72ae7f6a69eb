"""Device memory ownership through the C-ABI: a context whose memory comes
from PyTorch's caching allocator (nhdc_set_allocator) gives results bitwise
equal to one on the library's own hipMalloc, torch counts its footprint and
gets it back on destroy; destroying a context that a live batch holds defers
the release to the batch's destroy."""
import numpy as np
import pytest

from paper_2511_02021_amd.inputs import case as CS

pytestmark = pytest.mark.gpu

FIELDS = ("vn", "w", "rho", "pi", "theta_v", "pi_prev")


def _nhdc():
    from paper_2511_02021_amd import nhdc
    return nhdc


def test_torch_allocator_owns_the_context_memory_and_results_are_bitwise():
    import torch
    nhdc = _nhdc()
    c = CS.config_case(2, k=4, n_lev=30)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    d = nhdc.Dycore(c, allocator="torch")
    grown = torch.cuda.memory_allocated(0) - base
    nc, ne, N = c.grid.n_cells, c.grid.n_edges, c.n_lev
    # at least the state and the accumulators: vn, facc [N][ne]; w, wacc
    # [N+1][nc]; rho, pi, theta_v, pi_prev and the extrapolated Exner [N][nc]
    state_bytes = 8 * (2 * N * ne + 2 * (N + 1) * nc + 5 * N * nc)
    assert grown >= state_bytes, (grown, state_bytes)
    # FP64: every array an allocation of its own
    assert d.allocator.live > 30, d.allocator.live
    ref = nhdc.Dycore(c)  # hipMalloc
    assert torch.cuda.memory_allocated(0) - base == grown  # the library's own memory is not torch's
    for _ in range(3):
        d.step(c.dt, c.nsub)
        ref.step(c.dt, c.nsub)
    s, r = d.get_state(), ref.get_state()
    for f in FIELDS:
        assert np.array_equal(s[f], r[f]), f
    fa, ra = d.mass_flux(), ref.mass_flux()
    assert np.array_equal(fa[0], ra[0]) and np.array_equal(fa[1], ra[1])
    assert d.diag() == ref.diag()
    ref.close()
    alloc = d.allocator
    d.close()
    torch.cuda.synchronize()
    assert alloc.live == 0
    assert torch.cuda.memory_allocated(0) == base


def test_allocator_must_come_before_the_grid():
    nhdc = _nhdc()
    c = CS.config_case(1, k=2, n_lev=6)
    d = nhdc.Dycore(c)
    a = nhdc.TorchAllocator(0)
    with pytest.raises(nhdc.NhdcError) as e:
        d._check(d.L.nhdc_set_allocator(d.h, a.alloc, a.free, None))
    assert e.value.code == -5
    d.close()


def test_destroying_a_batched_context_defers_its_release():
    import torch
    nhdc = _nhdc()
    cases = [CS.config_case(2, k=3, n_lev=20), CS.config_case(2, k=3, n_lev=30, inst=1)]
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    # closed before any step, then the batch destroyed
    ds = [nhdc.Dycore(c, allocator="torch") for c in cases]
    b = nhdc.Batch(ds)
    ds[0].close()
    assert ds[0].allocator.live > 0  # still held by the batch
    b.close()
    assert ds[0].allocator.live == 0 and ds[1].allocator.live > 0
    ds[1].close()
    # closed while the batch keeps stepping it: the batch's results stay those
    # of the instances alone
    ds = [nhdc.Dycore(c, allocator="torch") for c in cases]
    b = nhdc.Batch(ds)
    b.step([c.dt for c in cases], 5, nsteps=1)
    h0 = ds[0].h  # stays valid: the batch holds the context
    ds[0].close()
    b.step([c.dt for c in cases], 5, nsteps=1)
    torch.cuda.synchronize()
    s1 = ds[1].get_state()
    alone = nhdc.Dycore(cases[1])
    for _ in range(2):
        alone.step(cases[1].dt, 5)
    r1 = alone.get_state()
    for f in FIELDS:
        assert np.array_equal(s1[f], r1[f]), f
    alone.close()
    # a destroyed context cannot join a new batch
    import ctypes as C
    hb = C.c_void_p()
    arr = (C.c_void_p * 1)(h0)
    assert nhdc.lib().nhdc_batch_create(C.byref(hb), arr, 1) == -5 and not hb.value
    b.close()
    ds[1].close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == base


@pytest.mark.parametrize("precision", ["mixed", "mixed_vn32"])
def test_arena_holds_every_array_with_every_option(precision):
    """The mixed forms take their arrays from one arena: with the upwind,
    damping, sponge and diffusion options (the most arrays) they all fit it,
    nothing falls back to an allocation of its own (two allocations in all:
    the arena and the launch descriptors), and the results are bitwise those
    of the library's own allocations."""
    nhdc = _nhdc()
    c = CS.with_params(CS.with_damping(CS.config_case(2, k=3, n_lev=20), sponge_base=20000.0),
                       upwind=1)
    d = nhdc.Dycore(c, precision=precision, allocator="torch")
    assert d.allocator.live == 2, d.allocator.live
    ref = nhdc.Dycore(c, precision=precision)
    for _ in range(2):
        d.step(c.dt, 5)
        ref.step(c.dt, 5)
    s, r = d.get_state(), ref.get_state()
    for f in FIELDS:
        assert np.array_equal(s[f], r[f]), (precision, f)
    d.close()
    ref.close()

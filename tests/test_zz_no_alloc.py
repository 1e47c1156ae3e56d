"""The allocation-free diagnostics entry point (snowlb_diag_noalloc) against snowlb_diag, through the
C ABI: bitwise the same FP64 sums and species invariant, on two calls in a row with the second on a
smaller lattice (fewer partials than the first left in the shared static scratch), in FP32 and 16-bit
storage; and inside a captured graph (where an allocation or a synchronisation would fail the
capture), replayed several times with eager steps in between."""
import gc

import numpy as np
import pytest

from paper_2101_07163_amd import snowlb as S
from paper_2101_07163_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def cfg_of(nx, ny, **kw):
    c = dict(W.COMMON)
    c.update(nx=nx, ny=ny, seed=(nx / 3, ny / 2, 6.0), w_init=1.0, U0=0.6)
    c.update(kw)
    return c


def noalloc(sim):
    out = torch.full((S.DIAG_COUNT,), float("nan"), dtype=torch.float64, device="cuda")
    S.snowlb_diag_noalloc(sim.ctx, out.data_ptr(), sim.stream)
    torch.cuda.current_stream().synchronize()
    return out.cpu().numpy()


def reference(sim):
    st, v = S.snowlb_diag(sim.ctx, sim.stream)
    assert st == S.OK
    return np.array(v)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_noalloc_matches_diag_on_two_calls_second_smaller(storage):
    # 1536^2 cells need the full 2048 partials; 96 x 80 needs 8, so the second call reads only the
    # partials it wrote itself while the scratch still holds the first call's
    big = S.Sim(cfg_of(1536, 1536, flow=1, inout=1, u_in=0.02, U_in=0.6), storage=storage).init().step(3)
    small = S.Sim(cfg_of(96, 80, flow=1, inout=1, u_in=0.02, U_in=0.6), storage=storage).init().step(5)
    for sim in (big, small):
        got, ref = noalloc(sim), reference(sim)
        print("  %d x %d %s: %s" % (sim.p.nx, sim.p.ny, storage, got))
        assert np.array_equal(got, ref)
        assert abs(got[8] / (ref[3] + 0.5 * sim.p.L_sat * ref[5]) - 1) < 1e-15


def test_noalloc_errors():
    sim = S.Sim(cfg_of(64, 64))
    out = torch.zeros(S.DIAG_COUNT, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SnowlbError) as e:
        S.snowlb_diag_noalloc(sim.ctx, out.data_ptr(), sim.stream)
    assert e.value.status == S.ESTATE
    sim.init()
    assert S.lib().snowlb_diag_noalloc(sim.ctx, None, None) == S.EINVAL


def test_noalloc_under_graph_capture():
    """Captured into a graph (capture fails on an allocation or a synchronisation), replayed three
    times with two eager steps between replays (the state returns to the same copy), each replay
    checked against snowlb_diag of the same state."""
    sim = S.Sim(cfg_of(200, 120, flow=1, inout=1, u_in=0.02, U_in=0.6)).init().step(4)
    noalloc(sim)  # first call on this device: the scratch address is looked up outside the capture
    out = torch.full((S.DIAG_COUNT,), float("nan"), dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    # Contexts of earlier tests that sit in reference cycles must not be destroyed during the capture:
    # their hipDeviceSynchronize / hipFree would invalidate a global-mode capture.  Collect them first
    # and keep the collector off while capturing.
    gc.collect()
    gc.disable()
    try:
        with torch.cuda.graph(g):
            S.snowlb_diag_noalloc(sim.ctx, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    finally:
        gc.enable()
    for _ in range(3):
        sim.step(2)
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), reference(sim))

"""Caller-owned device memory: after rtdm_bind_workspace every buffer of the
context lives in one torch allocation, and the results are bit-identical to
the same run on the library's own allocations; loading again moves the
buffers out first.  Contexts take their memory from PyTorch's caching
allocator by default (rtdm_set_allocator), with the same results."""

import gc

import numpy as np
import pytest

from paper_1404_5776_amd import rtdm, synth
from tests._common import gpu_context

pytestmark = pytest.mark.gpu


def _run(s, bind, use_graph=0, **opts):
    ctx = gpu_context(s, h_model=s.h_model, use_graph=use_graph, memory="library", **opts)
    n = ctx.bind_workspace() if bind else 0
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 3)
    rtdm.rtdm_step(ctx.h, s.dt, 4)
    out = (rtdm.rtdm_download(ctx.h, "K", s.b), rtdm.rtdm_dipole_trace(ctx.h), rtdm.rtdm_unitarity(ctx.h))
    if bind:
        # the geometry and ranges are fixed now; a second binding is refused
        with pytest.raises(rtdm.RtdmError):
            rtdm.rtdm_set_ranges(ctx.h, s.R_HS, s.R_P, s.R_K)
        with pytest.raises(rtdm.RtdmError):
            rtdm.rtdm_bind_workspace(ctx.h, ctx.workspace.data_ptr(), n)
    ctx.close()
    return out, n


@pytest.mark.parametrize("which,use_graph", [("cluster_b4", 0), ("lattice_b13", 1)])
def test_bound_workspace_gives_identical_results(which, use_graph):
    s = synth.config1() if which == "cluster_b4" else synth.diamond_lattice(
        (2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local", h_model="mulliken")
    (K0, tr0, u0), _ = _run(s, False, use_graph)
    (K1, tr1, u1), n = _run(s, True, use_graph)
    print(f"{which}: workspace {n / 2**20:.1f} MiB")
    assert n > (64 << 20)
    assert np.array_equal(K0, K1)
    assert np.array_equal(tr0[:, :6], tr1[:, :6])
    assert np.array_equal(u0, u1)


def test_too_small_or_foreign_workspace_is_refused():
    import torch
    s = synth.config1()
    ctx = gpu_context(s, memory="library")
    n = rtdm.rtdm_workspace_size(ctx.h)
    live = n - (64 << 20)               # the size includes a 64 MiB reserve
    small = torch.empty(live // 2, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_bind_workspace(ctx.h, small.data_ptr(), small.numel())
    assert e.value.code == -3          # RTDM_E_OOM
    host = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_bind_workspace(ctx.h, host.data_ptr(), n)
    # the context still works on its own allocations
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_step(ctx.h, s.dt, 2)
    ctx.close()


def test_workspace_without_reserve_suffices_for_inverse_and_steps():
    """A workspace of exactly the context's buffers (no reserve for
    temporaries): the inverse (whose b = 13 iteration keeps its column-major
    copy of S in a context buffer) and the steps allocate nothing more."""
    import torch
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=25, k0="local", h_model="mulliken")
    ref, _ = _run(s, False)
    ctx = gpu_context(s, h_model="mulliken", memory="library")
    live = rtdm.rtdm_workspace_size(ctx.h) - (64 << 20)
    ws = torch.empty(live, dtype=torch.uint8, device="cuda:0")
    rtdm.rtdm_bind_workspace(ctx.h, ws.data_ptr(), live)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 3)
    rtdm.rtdm_step(ctx.h, s.dt, 4)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    ctx.close()
    assert np.array_equal(K, ref[0])


def test_reload_in_a_bound_context_and_reserved_trace():
    """A bound context loads another system (its buffers move out of the
    workspace, the new system's set-up runs, a new workspace is bound) and
    then steps exactly as a fresh context does; with the trace reserved, the
    steps add no buffer (the context's memory total stays the same)."""
    a = synth.config1()
    b = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=27, k0="local", h_model="mulliken")
    ref, _ = _run(b, False)
    ctx = gpu_context(a, h_model="mulliken")
    ctx.bind_workspace()
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_step(ctx.h, a.dt, 2)
    ctx.load_system(b)                          # moves the buffers out of the region first
    assert ctx.workspace is None
    ctx.bind_workspace()
    rtdm.rtdm_reserve_trace(ctx.h, 4096)
    size0 = rtdm.rtdm_workspace_size(ctx.h)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, b.kappa)
    rtdm.rtdm_step(ctx.h, b.dt, 3)
    rtdm.rtdm_step(ctx.h, b.dt, 4)
    assert rtdm.rtdm_workspace_size(ctx.h) == size0
    K = rtdm.rtdm_download(ctx.h, "K", b.b)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    rtdm.rtdm_unbind_workspace(ctx.h)
    ctx.workspace = None
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_unbind_workspace(ctx.h)
    rtdm.rtdm_step(ctx.h, b.dt, 1)             # still steps on the library's own memory
    ctx.close()
    assert np.array_equal(K, ref[0])
    assert np.array_equal(tr[:, :6], ref[1][:, :6])


def test_torch_allocator_holds_the_context_and_gives_identical_results():
    """With the default memory="torch" every buffer is a PyTorch caching
    allocation: torch's allocated bytes grow by the context's total on load
    and fall back on close, and the run equals the one on hipMalloc memory."""
    import torch
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=28, k0="local", h_model="mulliken")
    ref, _ = _run(s, False)
    gc.collect()                    # contexts other tests left to the collector give their memory back now
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(0)
    ctx = gpu_context(s, h_model="mulliken")
    total = rtdm.rtdm_workspace_size(ctx.h) - (64 << 20)
    assert torch.cuda.memory_allocated(0) - before >= total
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 3)
    rtdm.rtdm_step(ctx.h, s.dt, 4)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    assert torch.cuda.memory_allocated(0) == before
    assert np.array_equal(K, ref[0])
    assert np.array_equal(tr[:, :6], ref[1][:, :6])


def test_torch_allocator_on_a_side_stream_with_graphs():
    """Steps issued on a torch side stream (captured graphs on it) with the
    context's memory from torch's caching allocator give the trace of steps
    on the default stream, and torch tensors allocated on that stream in
    between do not disturb them."""
    import torch
    s = synth.config1()
    ref, _ = _run(s, False)
    side = torch.cuda.Stream()
    ctx = gpu_context(s, h_model=s.h_model, use_graph=1, graph_steps=2)
    with torch.cuda.stream(side):
        rtdm.rtdm_build_inverse(ctx.h, side)
        rtdm.rtdm_apply_kick(ctx.h, s.kappa, side)
        rtdm.rtdm_step(ctx.h, s.dt, 3, side)
        junk = torch.randn(1 << 20, device="cuda:0")      # caching-allocator traffic on the same stream
        rtdm.rtdm_step(ctx.h, s.dt, 4, side)
        del junk
    side.synchronize()
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    assert np.array_equal(K, ref[0])
    assert np.array_equal(tr[:, :6], ref[1][:, :6])

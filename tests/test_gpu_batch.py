"""Batches of independent systems, captured step graphs and the launch-shape tuner.

A batch holds every (system, kick) pair as its own group of a block-diagonal
geometry; each group must follow the oracle's propagation of that system
with that kick (same 1e-10 bar and dipole rounding floor as single systems).
Graph replays must reproduce the eager steps bit for bit; tuning the launch
shape must not change any result bit.
"""

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, assert_charges, dipole_floor, gpu_charges, gpu_context, rel, small_clusters

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("h_model,b", [("fixed", 4), ("mulliken", 4), ("fixed", 13), ("mulliken", 13)])
def test_batch_of_clusters_with_xyz_kicks_matches_oracle(h_model, b):
    systems = small_clusters(b)
    kicks = [[(0.01, 0, 0), (0, 0.01, 0), (0, 0, 0.01)]] * len(systems)
    print(f"[gpu] batch of {len(systems)} b={b} clusters x 3 kicks, h_model={h_model}", flush=True)
    ctx = rtdm.Context(0, h_model=h_model)
    gptr = ctx.load_batch(systems, kicks)
    G = len(gptr) - 1
    assert G == 3 * len(systems)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick_groups(ctx.h, ctx.group_kicks)
    n_steps = 12
    rtdm.rtdm_step(ctx.h, 0.05, n_steps)
    gtr = rtdm.rtdm_group_trace(ctx.h, G)
    K = rtdm.rtdm_download(ctx.h, "K", b)
    rp, col = rtdm.rtdm_pattern(ctx.h, "K")
    xyz = ctx.batch_xyz
    q_all = gpu_charges(ctx, xyz.shape[0])
    ctx.close()
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    g = 0
    for sys_, ks in zip(systems, kicks):
        for kap in ks:
            a0 = gptr[g]
            # the oracle runs on the group's own (shifted) coordinates, the
            # inputs the batch was given
            st = O.setup(dataclasses.replace(sys_, xyz=xyz[a0:gptr[g + 1]]))
            ref = O.propagate(st, n_steps, 0.05, kap, h_model=h_model)
            sel = (rows >= a0) & (rows < gptr[g + 1])
            # this group's K blocks, in the oracle's pattern order (same relative order)
            assert rel(K[sel], ref.K.val) <= TOL
            dq = assert_charges(q_all[a0:gptr[g + 1]], ref.K, st.S)
            q0 = O.mulliken(O.kick(st.K0, st.xyz, kap), st.S)
            P0 = O.dipole(q0, st.xyz)
            induced = np.abs(ref.rows[:, 1:4] - P0).max()
            err = np.abs(gtr[:, g, :3] - ref.rows[:, 1:4]).max()
            assert err <= TOL * induced + dipole_floor(q0, st.xyz, dq)
            assert np.abs(gtr[:, g, 3] - ref.rows[:, 4]).max() <= TOL * abs(ref.rows[0, 4])
            g += 1


def _run(s, steps_chunks, use_graph, **opts):
    ctx = gpu_context(s, use_graph=int(use_graph), **opts)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    for n in steps_chunks:
        rtdm.rtdm_step(ctx.h, s.dt, n)
        rtdm.rtdm_observables(ctx.h)          # eager work and a synchronisation between replays
    out = (rtdm.rtdm_download(ctx.h, "K", s.b), rtdm.rtdm_dipole_trace(ctx.h))
    ctx.close()
    return out


@pytest.mark.parametrize("which", ["fixed_b4", "mulliken_b4", "mulliken_b4_1728", "mulliken_b13"])
@pytest.mark.parametrize("graph_steps", [1, 4])
def test_graph_replays_equal_eager_steps(which, graph_steps):
    """Steps replayed from captured graphs (one step per graph, or four: the
    calls of 4, 5 and 9 steps replay 4-step graphs and the one-step graph for
    the rest) repeat the eager steps bit for bit (the 1,728-atom lattice with
    row runs on the whole chip and the stored U^dagger)."""
    s = {"fixed_b4": synth.config1,
         "mulliken_b4": lambda: synth.diamond_lattice((3, 3, 3), 4, 10.0, 12.0, seed=22, h_model="mulliken"),
         "mulliken_b4_1728": lambda: synth.diamond_lattice((6, 6, 6), 4, 10.0, 12.0, seed=24, h_model="mulliken"),
         "mulliken_b13": lambda: synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local",
                                                       h_model="mulliken")}[which]()
    chunks = (3, 4, 5, 9)
    K_e, tr_e = _run(s, chunks, False, h_model=s.h_model)
    K_g, tr_g = _run(s, chunks, True, h_model=s.h_model, graph_steps=graph_steps)
    assert tr_e.shape == tr_g.shape == (sum(chunks), 7)
    for r in range(tr_e.shape[0]):                      # every replayed step
        assert np.array_equal(tr_e[r, :6], tr_g[r, :6]), r
    assert np.array_equal(K_e, K_g)


def test_autotune_keeps_results_bit_identical():
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=23, k0="local", h_model="mulliken")
    K_ref, tr_ref = _run(s, (4,), False, h_model="mulliken")
    ctx = gpu_context(s, h_model="mulliken")
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_step(ctx.h, s.dt, 1)                      # fills U, K for the timing runs
    wpb, tile = rtdm.rtdm_autotune(ctx.h)
    assert wpb in (4, 8, 16) and tile in (64, 256, 1024)
    ctx.load_system(s)                                   # fresh state, tuned shape kept
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 4)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    assert np.array_equal(K, K_ref)
    assert np.array_equal(tr[:, :6], tr_ref[:, :6])


def test_graph_recaptured_after_a_new_inverse():
    """step (graph) -> build_inverse -> step (graph) in one context repeats the
    eager sequence bit for bit: the inverse moves X between buffers and
    refreshes its column-major copy, so the captured step must be captured
    again rather than replayed."""
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=24, k0="local", h_model="mulliken")

    def run(use_graph):
        ctx = gpu_context(s, h_model="mulliken", use_graph=use_graph)
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_apply_kick(ctx.h, s.kappa)
        rtdm.rtdm_step(ctx.h, s.dt, 3)
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_step(ctx.h, s.dt, 3)
        out = (rtdm.rtdm_download(ctx.h, "K", s.b), rtdm.rtdm_dipole_trace(ctx.h))
        ctx.close()
        return out

    K_e, tr_e = run(0)
    K_g, tr_g = run(1)
    assert np.array_equal(K_e, K_g)
    assert np.array_equal(tr_e[:, :6], tr_g[:, :6])


def test_sixteen_step_graphs_equal_eager_steps_over_a_long_run():
    """The default 16 steps per graph over 100 steps of the 64-atom cluster
    (6 replays of the 16-step graph and 4 one-step replays)."""
    s = synth.config1()
    K_e, tr_e = _run(s, (100,), False)
    K_g, tr_g = _run(s, (100,), True)
    assert np.array_equal(K_e, K_g)
    assert np.array_equal(tr_e[:, :6], tr_g[:, :6])


def _members():
    """Contexts of differing kinds: b = 4 and b = 13 kick sets (fixed H: the
    first step builds U eagerly), a Mulliken-H b = 13 lattice with two
    corrector steps after the kick (eager too), and an ETRS b = 4 lattice of
    1,728 atoms (row runs on the whole chip, the stored U^dagger)."""
    kicks = [(0.01, 0, 0), (0, 0.01, 0), (0, 0, 0.01)]
    out = []
    for b in (4, 13):
        ctx = rtdm.Context(0, h_model="fixed", n_kicks=3)
        ctx.load_kick_sets(small_clusters(b), kicks)
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_apply_kicks(ctx.h, ctx.kick_vectors)
        out.append(ctx)
    s13 = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=25, k0="local", h_model="mulliken")
    s4 = synth.diamond_lattice((6, 6, 6), 4, 10.0, 12.0, seed=26, h_model="mulliken")
    for s, opts in ((s13, dict(h_model="mulliken", sc_steps=2, sc_iters=1)),
                    (s4, dict(h_model="mulliken", propagator="etrs"))):
        ctx = gpu_context(s, **opts)
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_apply_kick(ctx.h, s.kappa)
        out.append(ctx)
    return out


def _state(ctx):
    out = []
    for k in range(ctx.options.n_kicks):
        rtdm.rtdm_select_kick(ctx.h, k)
        out.append((rtdm.rtdm_download(ctx.h, "K", ctx.b), rtdm.rtdm_dipole_trace(ctx.h)[:, :6]))
    return out


def test_batch_step_equals_separate_steps():
    """One batch stepping four unlike contexts (4-step graphs, calls of 6 and
    11 steps: eager first steps, two and then one graph replay, an eager
    rest) leaves each context bit for bit where rtdm_step leaves it."""
    print("[gpu] batch of contexts vs separate rtdm_step calls", flush=True)
    dt, chunks = 0.05, (6, 11)
    ref = []
    for ctx in _members():
        for n in chunks:
            rtdm.rtdm_step(ctx.h, dt, n)
        ref.append(_state(ctx))
        ctx.close()
    ctxs = _members()
    bt = rtdm.rtdm_batch_create([c.h for c in ctxs], graph_steps=4)
    try:
        for n in chunks:
            rtdm.rtdm_batch_step(bt, dt, n)
            rtdm.rtdm_observables(ctxs[0].h)   # eager work and a synchronisation between calls
        got = [_state(c) for c in ctxs]
    finally:
        rtdm.rtdm_batch_destroy(bt)
    for i, (r, g) in enumerate(zip(ref, got)):
        for k, ((Kr, tr), (Kg, tg)) in enumerate(zip(r, g)):
            assert tr.shape == tg.shape == (sum(chunks), 6), (i, k)
            assert np.array_equal(Kr, Kg), (i, k)
            assert np.array_equal(tr, tg), (i, k)
    for c in ctxs:
        c.close()


def test_batch_step_refuses_unitarity_checks():
    s = synth.config1()
    ctx = gpu_context(s, unit_check_every=1)
    rtdm.rtdm_build_inverse(ctx.h)
    bt = rtdm.rtdm_batch_create([ctx.h])
    try:
        with pytest.raises(rtdm.RtdmError, match="unit_check_every"):
            rtdm.rtdm_batch_step(bt, s.dt, 2)
    finally:
        rtdm.rtdm_batch_destroy(bt)
        ctx.close()


def test_batch_of_one_context_equals_rtdm_step():
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=29, k0="local", h_model="mulliken")
    K_e, tr_e = _run(s, (7, 9), False, h_model="mulliken")
    ctx = gpu_context(s, h_model="mulliken")
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    bt = rtdm.rtdm_batch_create([ctx.h], graph_steps=3)
    try:
        for n in (7, 9):
            rtdm.rtdm_batch_step(bt, s.dt, n)
            rtdm.rtdm_observables(ctx.h)
        K = rtdm.rtdm_download(ctx.h, "K", s.b)
        tr = rtdm.rtdm_dipole_trace(ctx.h)
    finally:
        rtdm.rtdm_batch_destroy(bt)
        ctx.close()
    assert np.array_equal(K, K_e)
    assert np.array_equal(tr[:, :6], tr_e[:, :6])

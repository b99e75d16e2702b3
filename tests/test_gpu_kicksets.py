"""Kick sets: several K matrices stepped with one shared propagator per step.

A context created with n_kicks = 3 holds each system of a batch once; kick set
k starts from the ground state kicked along axis k.  With a fixed H the
propagator does not depend on K, so set k must repeat bit for bit what a
one-kick context of the same geometry does after kick k alone (the same
kernels on the same U), and every system's K, charges and traces in set k
must follow the oracle's propagation of that system with that kick (the
1e-10 bar and dipole rounding floor of the single-system tests).
"""

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, assert_charges, dipole_floor, gpu_charges, rel, small_clusters

pytestmark = pytest.mark.gpu

KICKS = [(0.01, 0.0, 0.0), (0.0, 0.01, 0.0), (0.0, 0.0, 0.01)]
DT, N_STEPS = 0.05, 12


def _read(ctx, b, G):
    n = ctx.batch_xyz.shape[0]
    return (rtdm.rtdm_download(ctx.h, "K", b), rtdm.rtdm_group_trace(ctx.h, G),
            rtdm.rtdm_dipole_trace(ctx.h), gpu_charges(ctx, n))


def _kick_sets(systems, use_graph):
    ctx = rtdm.Context(0, h_model="fixed", n_kicks=len(KICKS), use_graph=use_graph)
    gptr = ctx.load_kick_sets(systems, KICKS)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kicks(ctx.h, ctx.kick_vectors)
    for n in (5, N_STEPS - 5):
        rtdm.rtdm_step(ctx.h, DT, n)
    out = []
    for k in range(len(KICKS)):
        rtdm.rtdm_select_kick(ctx.h, k)
        out.append(_read(ctx, systems[0].b, len(gptr) - 1))
    rp, col = rtdm.rtdm_pattern(ctx.h, "K")
    xyz = ctx.batch_xyz
    ctx.close()
    return gptr, xyz, rp, out


def _one_kick(systems, kap):
    ctx = rtdm.Context(0, h_model="fixed")
    gptr = ctx.load_batch(systems, [[(0.0, 0.0, 0.0)]] * len(systems))
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, kap)
    for n in (5, N_STEPS - 5):
        rtdm.rtdm_step(ctx.h, DT, n)
    out = _read(ctx, systems[0].b, len(gptr) - 1)
    ctx.close()
    return out


@pytest.mark.parametrize("b", [4, 13])
def test_kick_sets_match_oracle_and_one_kick_runs(b):
    systems = small_clusters(b)
    print(f"[gpu] kick sets: {len(systems)} b={b} clusters x {len(KICKS)} kicks", flush=True)
    gptr, xyz, rp, sets = _kick_sets(systems, use_graph=0)
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    for k, kap in enumerate(KICKS):
        K, gtr, tr, q_all = sets[k]
        K1, gtr1, tr1, q1 = _one_kick(systems, kap)
        assert np.array_equal(K, K1), k
        assert np.array_equal(gtr, gtr1), k
        assert np.array_equal(tr[:, :6], tr1[:, :6]), k
        assert np.array_equal(q_all, q1), k
        for g, sys_ in enumerate(systems):
            a0, a1 = gptr[g], gptr[g + 1]
            st = O.setup(dataclasses.replace(sys_, xyz=xyz[a0:a1]))
            ref = O.propagate(st, N_STEPS, DT, kap, h_model="fixed")
            sel = (rows >= a0) & (rows < a1)
            assert rel(K[sel], ref.K.val) <= TOL
            dq = assert_charges(q_all[a0:a1], ref.K, st.S)
            q0 = O.mulliken(O.kick(st.K0, st.xyz, kap), st.S)
            P0 = O.dipole(q0, st.xyz)
            induced = np.abs(ref.rows[:, 1:4] - P0).max()
            assert np.abs(gtr[:, g, :3] - ref.rows[:, 1:4]).max() <= TOL * induced + dipole_floor(q0, st.xyz, dq)
            assert np.abs(gtr[:, g, 3] - ref.rows[:, 4]).max() <= TOL * abs(ref.rows[0, 4])


def test_kick_sets_on_row_runs_equal_one_kick_runs():
    """Two 1,728-atom b = 4 lattices: their products run over row runs of 16
    (not the split form of small systems) and W U^dagger reads the stored
    U^dagger, shared by the three kick sets; each set repeats a one-kick run
    bit for bit."""
    systems = [synth.diamond_lattice((6, 6, 6), 4, 10.0, 12.0, seed=36 + k, h_model="fixed") for k in range(2)]
    print("[gpu] kick sets: two 1728-atom b=4 lattices x 3 kicks", flush=True)
    gptr, _, _, sets = _kick_sets(systems, use_graph=1)
    for k, kap in enumerate(KICKS):
        K, gtr, tr, q_all = sets[k]
        K1, gtr1, tr1, q1 = _one_kick(systems, kap)
        assert np.array_equal(K, K1), k
        assert np.array_equal(gtr, gtr1), k
        assert np.array_equal(tr[:, :6], tr1[:, :6]), k
        assert np.array_equal(q_all, q1), k


def test_kick_sets_graph_replays_equal_eager_steps():
    systems = small_clusters(13)
    _, _, _, eager = _kick_sets(systems, use_graph=0)
    _, _, _, graph = _kick_sets(systems, use_graph=1)
    for k in range(len(KICKS)):
        for a, c in zip(eager[k][:2], graph[k][:2]):
            assert np.array_equal(a, c), k
        assert np.array_equal(eager[k][2][:, :6], graph[k][2][:, :6]), k


def test_kick_sets_refuse_a_k_dependent_propagator():
    with pytest.raises(rtdm.RtdmError):
        rtdm.Context(0, h_model="mulliken", n_kicks=3)
    ctx = rtdm.Context(0, h_model="fixed", n_kicks=2)
    systems = small_clusters(4)[:1]
    ctx.load_kick_sets(systems, KICKS[:2])
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_select_kick(ctx.h, 2)
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_set_state(ctx.h, np.zeros(2 + 3 * ctx.batch_xyz.shape[0]))
    ctx.close()


def test_kick_sets_with_unitarity_checks_record_every_set():
    """With unit_check_every = 2 the unitarity error of the shared propagator
    lands in the trace of every kick set (the same value), and each set's
    dipole rows still equal a one-kick run's."""
    systems = small_clusters(4)[:2]
    ctx = rtdm.Context(0, h_model="fixed", n_kicks=len(KICKS), unit_check_every=2)
    ctx.load_kick_sets(systems, KICKS)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kicks(ctx.h, ctx.kick_vectors)
    rtdm.rtdm_step(ctx.h, DT, 6)
    traces = []
    for k in range(len(KICKS)):
        rtdm.rtdm_select_kick(ctx.h, k)
        traces.append(rtdm.rtdm_dipole_trace(ctx.h))
    ctx.close()
    u = traces[0][:, 6]
    assert np.all(np.isfinite(u[1::2])) and np.all(np.isnan(u[0::2]))
    for k, kap in enumerate(KICKS):
        assert np.array_equal(traces[k][:, 6], u, equal_nan=True)
        one = rtdm.Context(0, h_model="fixed", unit_check_every=2)
        one.load_batch(systems, [[(0.0, 0.0, 0.0)]] * len(systems))
        rtdm.rtdm_build_inverse(one.h)
        rtdm.rtdm_apply_kick(one.h, kap)
        rtdm.rtdm_step(one.h, DT, 6)
        tr1 = rtdm.rtdm_dipole_trace(one.h)
        one.close()
        assert np.array_equal(traces[k][:, :6], tr1[:, :6]), k
        assert np.array_equal(traces[k][:, 6], tr1[:, 6], equal_nan=True), k

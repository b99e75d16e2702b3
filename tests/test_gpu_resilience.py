"""Checkpoint and resume, the unitarity monitor, non-finite detection and the
learned start's fallback, on the GPU.  Resume is bit-identical by
construction (same inputs, same kernels, same order), so it is compared with
array_equal."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import gpu_context

pytestmark = pytest.mark.gpu

FIELD = ((0.01, -0.005, 0.002), 0.2, 0.1)


def _lattice():
    return synth.diamond_lattice((3, 3, 3), 4, 10.0, 12.0, seed=22, h_model="mulliken")


@pytest.mark.parametrize("use_graph", [0, 1])
def test_resume_from_checkpoint_is_bit_identical(use_graph):
    s = _lattice()
    opts = dict(h_model="mulliken", propagator="etrs", sc_steps=8, sc_iters=2, use_graph=use_graph)
    # uninterrupted: 6 + 6 steps
    a = gpu_context(s, **opts)
    rtdm.rtdm_set_field(a.h, *FIELD)
    rtdm.rtdm_build_inverse(a.h)
    rtdm.rtdm_apply_kick(a.h, s.kappa)
    rtdm.rtdm_step(a.h, s.dt, 6)
    K6 = rtdm.rtdm_download(a.h, "K", s.b)
    state = rtdm.rtdm_get_state(a.h, s.n_atoms)
    rtdm.rtdm_step(a.h, s.dt, 6)
    tr_a = rtdm.rtdm_dipole_trace(a.h)
    K_a = rtdm.rtdm_download(a.h, "K", s.b)
    a.close()
    assert state[1] == 6 and abs(state[0] - 0.3) < 1e-15
    # resumed in a fresh context from (K, state)
    b = gpu_context(s, **opts)
    rtdm.rtdm_set_field(b.h, *FIELD)
    rtdm.rtdm_build_inverse(b.h)
    rtdm.rtdm_upload(b.h, "K", K6)
    rtdm.rtdm_set_state(b.h, state)
    rtdm.rtdm_step(b.h, s.dt, 6)
    tr_b = rtdm.rtdm_dipole_trace(b.h)
    K_b = rtdm.rtdm_download(b.h, "K", s.b)
    b.close()
    assert np.array_equal(tr_b[:, :6], tr_a[6:, :6])
    assert np.array_equal(K_b, K_a)


def test_unitarity_monitor_stops_an_unstable_step():
    s = synth.config1()
    ctx = gpu_context(s, unit_check_every=1, unit_tol=1e-6, taylor_order=2)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, 0.01, 2)                    # small steps pass
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    assert np.all(tr[:, 6] < 1e-6)
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_step(ctx.h, 1.5, 5)                 # a second-order series at dt 1.5 is far from unitary
    assert e.value.code == -6                         # RTDM_E_NUMERIC
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    assert tr.shape[0] == 3 and tr[-1, 6] > 1e-6      # stopped at the first bad check, row recorded
    ctx.close()


def test_non_finite_density_matrix_is_reported():
    s = synth.config1()
    ctx = gpu_context(s)
    st = O.setup(s)
    K = st.K0.val.copy()
    K[0, 0, 0] = np.nan
    rtdm.rtdm_upload(ctx.h, "K", K)
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_observables(ctx.h)
    assert e.value.code == -6
    ctx.close()


def test_poisoned_learned_start_falls_back_to_block_jacobi():
    s = _lattice()
    base = gpu_context(s)
    it0, _ = rtdm.rtdm_build_inverse(base.h)
    X0 = rtdm.rtdm_download(base.h, "X", s.b)
    base.close()
    ctx = gpu_context(s, inv_start="learned")
    n = rtdm.rtdm_mlp_params(ctx.h)[0]
    rng = np.random.default_rng(5)
    rtdm.rtdm_mlp_set_weights(ctx.h, (50.0 * rng.uniform(-1, 1, n)).astype(np.float32))
    it, res = rtdm.rtdm_build_inverse(ctx.h)
    total, fell_back = rtdm.rtdm_inverse_info(ctx.h)
    X = rtdm.rtdm_download(ctx.h, "X", s.b)
    ctx.close()
    assert fell_back == 1 and total > it0
    assert res <= 1e-10
    assert np.array_equal(X, X0)

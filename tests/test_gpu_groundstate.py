"""Ground state by truncated purification on the GPU against the oracle, and a
propagation started from it.  Same FP64 bar: K within 1e-10 relative, equal
iteration counts and branch sequences."""

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, assert_charges, dipole_floor, gpu_charges, gpu_context, rel

pytestmark = pytest.mark.gpu


def _systems(which):
    if which == "cluster_b4":
        return synth.config1()
    if which == "lattice_b4_R8":
        return synth.diamond_lattice((3, 3, 3), 4, 10.0, 8.0, seed=6, k0="local", h_model="mulliken")
    if which == "lattice_b13":
        return synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local", h_model="mulliken")
    raise KeyError(which)


@pytest.mark.parametrize("which", ["cluster_b4", "lattice_b4_R8", "lattice_b13"])
def test_ground_state_matches_oracle(which):
    s = _systems(which)
    n_occ = synth.n_occupied(s.n_atoms, s.b)
    ctx = gpu_context(s)
    rtdm.rtdm_build_inverse(ctx.h)
    it, idem, br = rtdm.rtdm_ground_state(ctx.h, n_occ)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    obs = rtdm.rtdm_observables(ctx.h)
    ctx.close()
    st = O.setup(s)
    X = O.hotelling(st.S, st.pat_p).X
    gs = O.ground_state(st.S, st.H0, X, st.pat_p, st.pat_k, n_occ)
    print(f"{which}: {it} iterations (oracle {gs.iters}), idempotency {idem:.2e}, K rel {rel(K, gs.K.val):.2e}, "
          f"Tr(KS) {obs[3]:.10f} of {n_occ}")
    assert it == gs.iters and br == gs.branches
    assert rel(K, gs.K.val) <= TOL
    assert np.array_equal(np.imag(K), np.zeros_like(np.imag(K)))
    assert abs(obs[3] - O.mulliken(gs.K, st.S).sum()) <= TOL * n_occ


def test_propagation_from_the_gpu_ground_state():
    s = _systems("lattice_b4_R8")
    n_occ = synth.n_occupied(s.n_atoms, s.b)
    ctx = gpu_context(s, h_model="mulliken")
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_ground_state(ctx.h, n_occ)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 10)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    q = gpu_charges(ctx, s.n_atoms)
    ctx.close()
    st = O.setup(s)
    X = O.hotelling(st.S, st.pat_p)
    gs = O.ground_state(st.S, st.H0, X.X, st.pat_p, st.pat_k, n_occ)
    st2 = dataclasses.replace(st, K0=gs.K)
    ref = O.propagate(st2, 10, s.dt, s.kappa, h_model="mulliken", X=X)
    q0 = O.mulliken(O.kick(gs.K, st.xyz, s.kappa), st.S)
    P0 = O.dipole(q0, st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    err = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max()
    print(f"dipole err {err:.2e} of induced {induced:.2e}; K rel {rel(K, ref.K.val):.2e}")
    assert rel(K, ref.K.val) <= TOL
    dq = assert_charges(q, ref.K, st.S)
    assert err <= TOL * induced + dipole_floor(q0, st.xyz, dq)


def test_ground_state_arguments_are_checked():
    s = _systems("cluster_b4")
    ctx = gpu_context(s)
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_ground_state(ctx.h, 128)           # no inverse yet
    rtdm.rtdm_build_inverse(ctx.h)
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_ground_state(ctx.h, -1.0)
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_ground_state(ctx.h, 128, tol=1e-30, max_iter=3)
    assert e.value.code == -5                        # RTDM_E_NOCONV
    ctx.close()

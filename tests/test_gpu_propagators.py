"""ETRS and fourth-order Magnus propagators, the self-consistent corrector,
the Gaussian field and the spectrum transform on the GPU against the oracle.

Same bar as the plain path: matrices within 1e-10 relative (Frobenius),
dipole traces within 1e-10 of the induced signal plus the rounding floor of
the dipole sum, Tr(KS) within 1e-10 relative.  Spectra: the transform is a
weighted sum of that trace, so alpha_jj(w) may differ by the trace's bound
times sum_k exp(-gamma t_k) dt / |F[E_j](w)|.
"""

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, assert_charges, dipole_floor, gpu_charges, gpu_context, rel

pytestmark = pytest.mark.gpu

FIELD = O.Field((0.02, -0.01, 0.005), 0.2, 0.1)


def _systems(which):
    if which == "cluster_b4":
        return synth.config1()
    if which == "lattice_b4":
        return synth.diamond_lattice((3, 3, 3), 4, 10.0, 12.0, seed=22, h_model="mulliken")
    if which == "lattice_b13":
        return synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local", h_model="mulliken")
    raise KeyError(which)


def _run_gpu(s, n_steps, kappa, field=None, chunks=None, **opts):
    ctx = gpu_context(s, h_model=s.h_model, **opts)
    if field is not None:
        rtdm.rtdm_set_field(ctx.h, field.E0, field.t0, field.sigma)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, kappa)
    p0 = rtdm.rtdm_observables(ctx.h)[:3]
    for n in (chunks or (n_steps,)):
        rtdm.rtdm_step(ctx.h, s.dt, n)
    out = dict(trace=rtdm.rtdm_dipole_trace(ctx.h), K=rtdm.rtdm_download(ctx.h, "K", s.b),
               U=rtdm.rtdm_download(ctx.h, "U", s.b), q=gpu_charges(ctx, s.n_atoms), p0=p0, ctx=ctx)
    return out


def _compare(s, g, ref, st, kappa):
    q0 = O.mulliken(O.kick(st.K0, st.xyz, kappa), st.S)
    P0 = O.dipole(q0, st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    err = np.abs(g["trace"][:, 1:4] - ref.rows[:, 1:4]).max()
    print(f"K rel {rel(g['K'], ref.K.val):.2e}  U rel {rel(g['U'], ref.U.val):.2e}  "
          f"dipole err {err:.2e} of induced {induced:.2e}")
    assert rel(g["K"], ref.K.val) <= TOL
    assert rel(g["U"], ref.U.val) <= TOL
    dq = assert_charges(g["q"], ref.K, st.S)
    assert err <= TOL * induced + dipole_floor(q0, st.xyz, dq)
    assert np.abs(g["trace"][:, 4] - ref.rows[:, 4]).max() <= TOL * np.abs(ref.rows[:, 4]).max()


@pytest.mark.parametrize("which", ["cluster_b4", "lattice_b4", "lattice_b13"])
@pytest.mark.parametrize("kind", ["etrs", "m4"])
def test_propagator_matches_oracle(kind, which):
    s = _systems(which)
    n = 4
    g = _run_gpu(s, n, s.kappa, propagator=kind)
    g["ctx"].close()
    st = O.setup(s)
    ref = O.propagate(st, n, s.dt, s.kappa, h_model=s.h_model, propagator=kind)
    _compare(s, g, ref, st, s.kappa)


@pytest.mark.parametrize("which", ["cluster_b4", "lattice_b13"])
@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_gaussian_field_matches_oracle(kind, which):
    s = _systems(which)
    n = 6
    g = _run_gpu(s, n, (0.0, 0.0, 0.0), field=FIELD, chunks=(2, 4), propagator=kind)
    g["ctx"].close()
    st = O.setup(s)
    ref = O.propagate(st, n, s.dt, (0, 0, 0), h_model=s.h_model, propagator=kind, field=FIELD)
    _compare(s, g, ref, st, (0, 0, 0))


@pytest.mark.parametrize("which", ["lattice_b4", "lattice_b13"])
@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_self_consistent_corrector_matches_oracle(kind, which):
    s = _systems(which)
    n, sc_steps, sc_iters = 5, 3, 2
    g = _run_gpu(s, n, s.kappa, propagator=kind, sc_steps=sc_steps, sc_iters=sc_iters)
    g["ctx"].close()
    st = O.setup(s)
    ref = O.propagate(st, n, s.dt, s.kappa, h_model="mulliken", propagator=kind, sc_steps=sc_steps,
                      sc_iters=sc_iters)
    _compare(s, g, ref, st, s.kappa)


@pytest.mark.parametrize("kind", ["em", "m4"])
def test_graph_with_field_and_corrector_equals_eager(kind):
    s = _systems("lattice_b4")
    res = []
    for use_graph in (0, 1):
        g = _run_gpu(s, 9, s.kappa, field=FIELD, chunks=(3, 2, 4), propagator=kind, sc_steps=2, sc_iters=2,
                     use_graph=use_graph)
        g["ctx"].close()
        res.append(g)
    for r in range(9):
        assert np.array_equal(res[0]["trace"][r, :6], res[1]["trace"][r, :6]), r
    assert np.array_equal(res[0]["K"], res[1]["K"])


def _alpha_bound(q0, xyz, rows, P0, dt, gamma, FE):
    """Bound on |alpha_gpu - alpha_oracle| per (w, j) from the trace's bound."""
    induced = np.abs(rows[:, 1:4] - P0).max()
    err_p = TOL * induced + dipole_floor(q0, xyz)
    t = dt * np.arange(rows.shape[0] + 1)
    w = (np.exp(-gamma * t) * dt).sum()
    with np.errstate(divide="ignore"):
        return err_p * w / np.abs(FE)


def _check_spectrum(alpha, sw, a_ref, s_ref, bound, om, dirs):
    for j in dirs:
        d = np.abs(alpha[:, j] - a_ref[:, j])
        print(f"alpha_{j}{j}: max {np.abs(a_ref[:, j]).max():.3e}, diff {d.max():.2e}, "
              f"bound {bound[:, j].min():.2e}..{bound[:, j].max():.2e}")
        assert np.all(d <= bound[:, j] + 1e-12 * np.abs(a_ref[:, j]).max())
    sb = 2 * om / np.pi * sum(bound[:, j] for j in dirs) / 3
    assert np.all(np.abs(sw - s_ref) <= sb + 1e-12 * np.abs(s_ref).max())


def test_kick_spectrum_matches_oracle():
    s = _systems("cluster_b4")
    n = 200
    kap = (1e-3, 0.0, 0.0)
    g = _run_gpu(s, n, kap)
    om = np.linspace(0.05, 2.5, 64)
    alpha, sw = rtdm.rtdm_spectrum(g["ctx"].h, g["p0"], om, 0.05, kappa=kap)
    g["ctx"].close()
    st = O.setup(s)
    ref = O.propagate(st, n, s.dt, kap)
    P0 = O.dipole(O.mulliken(O.kick(st.K0, st.xyz, kap), st.S), st.xyz)
    a_ref, s_ref = O.spectrum(ref.rows[:, 1:4], P0, s.dt, None, np.asarray(kap), 0.05, om)
    assert np.all(np.isnan(alpha[:, 1:])) and np.all(np.isnan(a_ref[:, 1:]))
    q0 = O.mulliken(O.kick(st.K0, st.xyz, kap), st.S)
    FE = np.broadcast_to(-np.asarray(kap), (om.size, 3))
    bound = _alpha_bound(q0, st.xyz, ref.rows, P0, s.dt, 0.05, FE)
    _check_spectrum(alpha, sw, a_ref, s_ref, bound, om, [0])


def test_field_spectrum_matches_oracle():
    s = _systems("cluster_b4")
    n = 120
    f = O.Field((1e-3, 5e-4, 0.0), 0.3, 0.1)
    g = _run_gpu(s, n, (0, 0, 0), field=f)
    om = np.linspace(0.05, 2.5, 40)
    alpha, sw = rtdm.rtdm_spectrum(g["ctx"].h, g["p0"], om, 0.1)
    g["ctx"].close()
    st = O.setup(s)
    ref = O.propagate(st, n, s.dt, (0, 0, 0), field=f)
    P0 = O.dipole(O.mulliken(st.K0, st.S), st.xyz)
    E = np.array([f.at(k * s.dt) for k in range(n + 1)])
    a_ref, s_ref = O.spectrum(ref.rows[:, 1:4], P0, s.dt, E, None, 0.1, om)
    assert np.all(np.isnan(alpha[:, 2]))
    t = s.dt * np.arange(n + 1)
    FE = (np.exp((1j * om[:, None] - 0.1) * t[None, :]) * s.dt) @ E
    bound = _alpha_bound(O.mulliken(st.K0, st.S), st.xyz, ref.rows, P0, s.dt, 0.1, FE)
    _check_spectrum(alpha, sw, a_ref, s_ref, bound, om, [0, 1])


def test_batched_xyz_kicks_give_the_strength_function():
    """x, y and z kicks of one cluster as three groups of one batch: the
    per-group spectra equal the oracle's and combine to S(w)."""
    s = synth.random_cluster(40, 4, 8.0, 12.0, 33, k0="exact")
    kap = 1e-3
    kicks = [[(kap, 0, 0), (0, kap, 0), (0, 0, kap)]]
    ctx = rtdm.Context(0)
    gptr = ctx.load_batch([s], kicks)
    rtdm.rtdm_build_inverse(ctx.h)
    n = 100
    xyz = ctx.batch_xyz
    st_groups, P0s = [], []
    for gi in range(3):
        sys_g = dataclasses.replace(s, xyz=xyz[gptr[gi]:gptr[gi + 1]])
        st = O.setup(sys_g)
        st_groups.append(st)
        P0s.append(O.dipole(O.mulliken(O.kick(st.K0, st.xyz, kicks[0][gi]), st.S), st.xyz))
    rtdm.rtdm_apply_kick_groups(ctx.h, ctx.group_kicks)
    rtdm.rtdm_step(ctx.h, s.dt, n)
    om = np.linspace(0.05, 2.5, 50)
    alphas = []
    for gi in range(3):
        a, _ = rtdm.rtdm_spectrum(ctx.h, P0s[gi], om, 0.05, kappa=kicks[0][gi], group=gi)
        alphas.append(a[:, gi])
    ctx.close()
    sw = 2 * om / np.pi * np.imag(sum(alphas) / 3)
    s_ref, s_bound = 0, 0
    for gi in range(3):
        st = st_groups[gi]
        ref = O.propagate(st, n, s.dt, kicks[0][gi])
        a_ref, _ = O.spectrum(ref.rows[:, 1:4], P0s[gi], s.dt, None, np.asarray(kicks[0][gi]), 0.05, om)
        q0 = O.mulliken(O.kick(st.K0, st.xyz, kicks[0][gi]), st.S)
        FE = np.broadcast_to(-np.asarray(kicks[0][gi]), (om.size, 3))
        bound = _alpha_bound(q0, st.xyz, ref.rows, P0s[gi], s.dt, 0.05, FE)
        assert np.all(np.abs(alphas[gi] - a_ref[:, gi]) <= bound[:, gi] + 1e-12 * np.abs(a_ref[:, gi]).max())
        s_ref = s_ref + 2 * om / np.pi * np.imag(a_ref[:, gi] / 3)
        s_bound = s_bound + 2 * om / np.pi * bound[:, gi] / 3
    assert np.all(np.abs(sw - s_ref) <= s_bound + 1e-12 * np.abs(s_ref).max())


def test_field_and_propagator_arguments_are_checked():
    s = _systems("cluster_b4")
    with pytest.raises(rtdm.RtdmError):
        rtdm.Context(0, propagator=7)
    with pytest.raises(rtdm.RtdmError):
        rtdm.Context(0, propagator="m4", precision="fp32")
    ctx = gpu_context(s)
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_set_field(ctx.h, (1.0, 0, 0), 0.0, 0.0)
    with pytest.raises(rtdm.RtdmError):
        rtdm.rtdm_spectrum(ctx.h, (0, 0, 0), np.ones(3), 0.1, kappa=(1e-3, 0, 0))   # no steps yet
    ctx.close()

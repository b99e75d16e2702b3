"""GPU path vs the oracle, element by element, through the C ABI.

Sizes are small enough for the oracle to finish in seconds, yet span many
output blocks (ragged against the four-wave workgroups and the 16-wide MFMA
tiles: b = 1, 4, 13, 16 and atom counts that are not multiples of 4).
The FP64 bar is 1e-10 relative (Frobenius for matrices, max-norm relative to
the signal for traces); integer results (patterns, triple counts, iteration
counts) must be identical.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, assert_charges, assert_same_pattern, dipole_floor, gpu_charges, gpu_context, rel

pytestmark = pytest.mark.gpu


def _cluster(n, b, R_HS, R_K, seed, R_P=None, **kw):
    rng = np.random.default_rng(seed)
    xyz = synth.cluster_positions(n, rng)
    return synth.build_system(f"cl{n}_b{b}", xyz, b, R_HS, R_K, seed, R_P=R_P, **kw)


SYSTEMS = {
    "b4_distinct_ranges": lambda: _cluster(45, 4, 6.0, 7.5, 101, R_P=9.0),
    "b13_shared_ranges": lambda: _cluster(37, 13, 6.0, 8.0, 102),
    "b1": lambda: _cluster(50, 1, 6.0, 8.0, 103, R_P=7.0),
    "b16": lambda: _cluster(21, 16, 6.0, 8.0, 104),
}


@pytest.fixture(scope="module", params=sorted(SYSTEMS))
def system(request):
    s = SYSTEMS[request.param]()
    return s, O.setup(s)


@pytest.fixture
def case(system):
    s, st = system
    ctx = gpu_context(s)
    yield s, st, ctx
    ctx.close()


def _random(pat: O.Pattern, b, seed, cplx):
    r = pat.rows()
    return synth.random_blocks(r, pat.col, b, seed, cplx)


def test_patterns_match_oracle(case):
    s, st, ctx = case
    assert_same_pattern(ctx, "S", st.pat_hs)
    assert_same_pattern(ctx, "X", st.pat_p)
    assert_same_pattern(ctx, "K", st.pat_k)


@pytest.mark.parametrize("kind", ["XH", "AT", "UK", "WU", "SX", "UVreal", "UKalpha"])
def test_product_matches_oracle(case, kind):
    s, st, ctx = case
    b = s.b
    h = ctx.h
    pp, ph, pk = st.pat_p, st.pat_hs, st.pat_k
    spec = {
        # kind: (C slot, A slot, B slot, op_a, op_b, alpha, (A pattern, A complex), (B pattern, B complex), C pattern)
        "XH": ("A", "X", "H", 0, 0, 1.0, (pp, False), (ph, False), pp),
        "AT": ("U", "A", "X", 0, 0, 0.37, (pp, False), (pp, False), pp),
        "UK": ("W", "U", "K", 0, 0, 1.0, (pp, True), (pk, True), pk),
        "WU": ("K", "W", "U", 0, 1, 1.0, (pk, True), (pp, True), pk),
        "SX": ("A", "S", "X", 0, 0, 1.0, (ph, False), (pp, False), pp),
        "UVreal": ("U", "X", "A", 1, 0, 1.0, (pp, False), (pp, False), pp),
        "UKalpha": ("W", "U", "K", 0, 0, 0.3 - 0.7j, (pp, True), (pk, True), pk),
    }[kind]
    Cs, As, Bs, oa, ob, alpha, (pa, ca), (pb, cb), pc = spec
    a = _random(pa, b, 11, ca)
    bm = _random(pb, b, 12, cb)
    rtdm.rtdm_upload(h, As, a)
    rtdm.rtdm_upload(h, Bs, bm)
    rtdm.rtdm_multiply(h, Cs, As, Bs, oa, ob, alpha)
    got = rtdm.rtdm_download(h, Cs, b)
    A = O.BSM(pa, b, a.astype(np.complex128))
    B = O.BSM(pb, b, bm.astype(np.complex128))
    want, trip = O.spgemm(A, B, pc, alpha=alpha, op_a=oa, op_b=ob)
    assert rel(got, want.val) <= TOL
    assert np.abs(got - want.val).max() <= TOL * np.abs(want.val).max()


def test_schedule_triples_match_oracle(case):
    s, st, ctx = case
    b = s.b
    z = lambda p: O.zeros(p, b)
    kinds = {"XH": (z(st.pat_p), z(st.pat_hs), st.pat_p, 0, 0),
             "AT": (z(st.pat_p), z(st.pat_p), st.pat_p, 0, 0),
             "UK": (z(st.pat_p), z(st.pat_k), st.pat_k, 0, 0),
             "WU": (z(st.pat_k), z(st.pat_p), st.pat_k, 0, 1),
             "SX": (z(st.pat_hs), z(st.pat_p), st.pat_p, 0, 0),
             "UV": (z(st.pat_p), z(st.pat_p), st.pat_p, 1, 0)}
    for k, (A, B, pc, oa, ob) in kinds.items():
        _, trip = O.spgemm(A, B, pc, op_a=oa, op_b=ob)
        outs, t = rtdm.rtdm_schedule_stats(ctx.h, k)
        assert (outs, t) == (pc.nnzb, trip), k


def test_inverse_matches_oracle(case):
    s, st, ctx = case
    it, r = rtdm.rtdm_build_inverse(ctx.h)
    ref = O.hotelling(st.S, st.pat_p)
    assert it == ref.iters
    assert abs(r - ref.residuals[-1]) <= 1e-6 * ref.residuals[-1] + 1e-15
    X = rtdm.rtdm_download(ctx.h, "X", s.b)
    assert rel(X, ref.X.val) <= TOL
    err = rtdm.rtdm_inverse_error(ctx.h)
    want = O.inverse_error(ref.X, st.S, st.pat_p)
    np.testing.assert_allclose(err, want, rtol=1e-6, atol=1e-16)


def test_cold_and_previous_starts_match_oracle():
    s = _cluster(40, 4, 6.0, 8.0, 105)
    st = O.setup(s)
    ctx = gpu_context(s, inv_start="cold")
    it, _ = rtdm.rtdm_build_inverse(ctx.h)
    ref = O.hotelling(st.S, st.pat_p, X0=O.cold_start(st.S, st.pat_p))
    assert it == ref.iters and not ref.fell_back
    assert rel(rtdm.rtdm_download(ctx.h, "X", s.b), ref.X.val) <= TOL
    ctx.close()
    # a diverging previous guess falls back to the block-Jacobi start
    ctx = gpu_context(s, inv_start="previous")
    bad = O.identity(st.pat_p, s.b)
    bad.val *= 5.0
    rtdm.rtdm_upload(ctx.h, "X", bad.val.real.copy())
    it, _ = rtdm.rtdm_build_inverse(ctx.h)
    ref = O.hotelling(st.S, st.pat_p, X0=bad)
    assert ref.fell_back and it == ref.iters
    assert rel(rtdm.rtdm_download(ctx.h, "X", s.b), ref.X.val) <= TOL
    ctx.close()


def test_kick_and_observables_match_oracle(case):
    s, st, ctx = case
    kappa = (0.03, -0.02, 0.01)
    rtdm.rtdm_upload_coo(ctx.h, "K", s.K0.rows, s.K0.cols, s.K0.data)
    rtdm.rtdm_apply_kick(ctx.h, kappa)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    Kref = O.kick(st.K0, st.xyz, kappa)
    assert rel(K, Kref.val) <= 1e-14
    obs = rtdm.rtdm_observables(ctx.h)
    q = O.mulliken(Kref, st.S)
    P = O.dipole(q, st.xyz)
    np.testing.assert_allclose(obs[:3], P, rtol=0, atol=TOL * np.abs(P).max() + dipole_floor(q, st.xyz))
    assert abs(obs[3] - q.sum()) <= TOL * abs(q.sum())


def _propagation_parity(s, n_steps, unit_every=0, check_unitarity=True, **opts):
    st = O.setup(s)
    ctx = gpu_context(s, h_model=s.h_model, unit_check_every=unit_every, **opts)
    it, _ = rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    obs0 = rtdm.rtdm_observables(ctx.h)
    rtdm.rtdm_step(ctx.h, s.dt, n_steps)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    U = rtdm.rtdm_download(ctx.h, "U", s.b)
    unit = rtdm.rtdm_unitarity(ctx.h) if check_unitarity else None
    q = gpu_charges(ctx, s.n_atoms)
    ctx.close()
    ref = O.propagate(st, n_steps, s.dt, s.kappa, h_model=s.h_model)
    dq = assert_charges(q, ref.K, st.S)
    assert it == ref.inverse.iters
    q0 = O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S)
    P0 = O.dipole(q0, st.xyz)
    np.testing.assert_allclose(obs0[:3], P0, rtol=0, atol=TOL * np.abs(P0).max() + dipole_floor(q0, st.xyz))
    floor = dipole_floor(q0, st.xyz, dq)
    assert tr.shape == (n_steps, 7)
    np.testing.assert_allclose(tr[:, 0], ref.rows[:, 0], rtol=1e-14)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    err = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max()
    print(f"dipole error {err:.2e}, induced {induced:.2e}, rounding floor {floor:.2e}")
    assert err <= TOL * induced + floor
    assert np.abs(tr[:, 4] - ref.rows[:, 4]).max() <= TOL * np.abs(ref.rows[:, 4]).max()
    np.testing.assert_allclose(tr[:, 5], ref.rows[:, 5], rtol=1e-4, atol=1e-15)
    assert rel(K, ref.K.val) <= TOL
    assert rel(U, ref.U.val) <= TOL
    if not check_unitarity:
        return tr
    ur = O.unitarity(ref.U, st.S, st.pat_p)
    np.testing.assert_allclose(unit, ur, rtol=1e-6, atol=1e-16)
    if unit_every:
        np.testing.assert_allclose(tr[n_steps - 1, 6], ur[0], rtol=1e-6)
        assert np.isnan(tr[0, 6]) or unit_every == 1
    return tr


def test_config1_full_run_matches_oracle():
    """The 64-atom cluster, fixed H, all 100 steps."""
    _propagation_parity(synth.config1(), 100, unit_every=25)


@pytest.mark.parametrize("xh_every_step", [0, 1])
def test_mulliken_b13_lattice_matches_oracle(xh_every_step):
    """Both ways of forming A: A0 + X D (default) and the full X H product."""
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local", h_model="mulliken")
    _propagation_parity(s, 5, unit_every=5, xh_every_step=xh_every_step)


def test_mulliken_b13_lattice512_matches_oracle():
    """512 atoms (4 x 4 x 4 cells) at the bench ranges: 29 % of the atom pairs
    are kept, so the cut-off truncates every product (the 64-atom lattice
    keeps 94 %).  Inverse plus two steps; the oracle needs about a minute."""
    s = synth.diamond_lattice((4, 4, 4), 13, 10.0, 16.0, seed=23, k0="local", h_model="mulliken")
    _propagation_parity(s, 2, check_unitarity=False)


@pytest.mark.parametrize("xh_every_step", [0, 1])
def test_mulliken_b4_lattice_matches_oracle(xh_every_step):
    s = synth.diamond_lattice((4, 4, 4), 4, 10.0, 12.0, seed=22, h_model="mulliken")
    _propagation_parity(s, 20, unit_every=10, xh_every_step=xh_every_step)


def test_b4_lattice_on_row_runs_matches_oracle():
    """1,728 atoms at b = 4: enough outputs (about 10,000 runs of 16) for the
    products to run over row runs on the whole chip rather than the split
    form of small systems, with W U^dagger reading the stored U^dagger."""
    s = synth.diamond_lattice((6, 6, 6), 4, 10.0, 12.0, seed=35, h_model="mulliken")
    _propagation_parity(s, 4, unit_every=4)


def test_taylor_order_option_matches_oracle():
    s = _cluster(30, 4, 6.0, 8.0, 106, h_model="fixed")
    st = O.setup(s)
    for p in (1, 2, 6):
        ctx = gpu_context(s, taylor_order=p)
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_apply_kick(ctx.h, s.kappa)
        rtdm.rtdm_step(ctx.h, 0.1, 3)
        K = rtdm.rtdm_download(ctx.h, "K", s.b)
        ctx.close()
        ref = O.propagate(st, 3, 0.1, s.kappa, p=p)
        assert rel(K, ref.K.val) <= TOL, p


def test_runs_are_bit_identical():
    s = synth.config1()
    out = []
    for _ in range(2):
        ctx = gpu_context(s)
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_apply_kick(ctx.h, s.kappa)
        rtdm.rtdm_step(ctx.h, s.dt, 10)
        out.append((rtdm.rtdm_download(ctx.h, "K", s.b), rtdm.rtdm_dipole_trace(ctx.h)))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1][:, :6], out[1][1][:, :6])


def test_hermitisation_is_exact():
    s = synth.config1()
    ctx = gpu_context(s)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 3)
    K = rtdm.rtdm_download(ctx.h, "K", s.b)
    rp, col = rtdm.rtdm_pattern(ctx.h, "K")
    ctx.close()
    pat = O.Pattern(s.n_atoms, s.R_K, rp, col)
    t = pat.transpose_index()
    assert np.array_equal(K, np.conj(np.transpose(K[t], (0, 2, 1))))


def test_error_paths():
    s = _cluster(20, 4, 6.0, 8.0, 107)
    ctx = rtdm.Context(0)
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_set_ranges(ctx.h, 6.0, 0.0, 8.0)
    assert e.value.code == -2                                   # geometry first
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_set_geometry(ctx.h, s.xyz, np.r_[s.nbf[:-1], 6])
    assert e.value.code == -7                                   # mixed sizes padded to neither 4 nor 13
    ctx.load_system(s)
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_step(ctx.h, 0.05, 1)
    assert e.value.code == -2                                   # no inverse yet
    far = int(np.argmax(np.linalg.norm(s.xyz - s.xyz[0], axis=1)))
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_upload_coo(ctx.h, "S", [0], [far], np.zeros((1, 4, 4)))
    assert e.value.code == -1                                   # block outside the cut-off
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_upload(ctx.h, "S", np.ones((O.setup(s).pat_hs.nnzb, 4, 4)) * 1j)
    assert e.value.code == -7                                   # complex data into a real slot
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_multiply(ctx.h, "K", "S", "H", 0, 0)
    assert e.value.code == -7                                   # no such product kind
    ctx.close()
    # a negative-definite "overlap" makes the cold-start iteration diverge
    ctx = rtdm.Context(0, inv_start="cold").load_system(s)
    rtdm.rtdm_upload_coo(ctx.h, "S", s.S.rows, s.S.cols, -s.S.data)
    with pytest.raises(rtdm.RtdmError) as e:
        rtdm.rtdm_build_inverse(ctx.h)
    assert e.value.code == -5
    ctx.close()

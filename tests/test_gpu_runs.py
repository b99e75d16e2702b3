"""Row runs of the block products against the oracle.

The step products (X H, A tau, U K, W U^dagger) at b = 13 can compute several
output blocks of one row per wave, sharing the left operand's loads; the run
length is chosen per context (RTDM_RUN_REAL for the real products: 1 to 4
or 8; RTDM_RUN_CPLX for the complex ones: 1 to 4).  At b = 4 the products
run over runs of 16 outputs (RTDM_RUN_B4=16) or per-output lists
(RTDM_RUN_B4=1).  Only the order of the contraction sums differs, so every
run length must meet the FP64 bar against the oracle, and agree with the
single-output kernels to a few ulps.  The systems have rows whose lengths
are not multiples of the run length, so short runs (absent outputs) are
exercised.
"""

import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, assert_charges, dipole_floor, gpu_charges, gpu_context, rel

pytestmark = pytest.mark.gpu

RUNS = [(1, 1), (2, 2), (3, 3), (4, 4), (8, 4), (8, 2)]
N_STEPS = 4


def _lattice():
    return synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=31, k0="local", h_model="mulliken")


def _cluster():
    rng = np.random.default_rng(32)
    xyz = synth.cluster_positions(37, rng)
    return synth.build_system("cl37_b13", xyz, 13, 6.0, 8.0, 32, h_model="mulliken")


SYSTEMS = {"lattice64_b13": _lattice, "cluster37_b13": _cluster}


@pytest.fixture(scope="module", params=sorted(SYSTEMS))
def reference(request):
    s = SYSTEMS[request.param]()
    st = O.setup(s)
    ref = O.propagate(st, N_STEPS, s.dt, s.kappa, h_model=s.h_model)
    return s, st, ref


def _run(s, run_real, run_cplx, run_b4=16, **opts):
    old = {k: os.environ.get(k) for k in ("RTDM_RUN_REAL", "RTDM_RUN_CPLX", "RTDM_RUN_B4")}
    os.environ["RTDM_RUN_REAL"] = str(run_real)
    os.environ["RTDM_RUN_CPLX"] = str(run_cplx)
    os.environ["RTDM_RUN_B4"] = str(run_b4)
    try:
        ctx = gpu_context(s, h_model=s.h_model, **opts)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    try:
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_apply_kick(ctx.h, s.kappa)
        rtdm.rtdm_step(ctx.h, s.dt, N_STEPS)
        return rtdm.rtdm_download(ctx.h, "K", s.b), rtdm.rtdm_dipole_trace(ctx.h), gpu_charges(ctx, s.n_atoms)
    finally:
        ctx.close()


@pytest.mark.parametrize("run_real,run_cplx", RUNS)
def test_row_runs_match_oracle(reference, run_real, run_cplx):
    s, st, ref = reference
    K, tr, q = _run(s, run_real, run_cplx, use_graph=0)
    q0 = O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S)
    P0 = O.dipole(q0, st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    err = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max()
    print(f"runs {run_real}/{run_cplx}: K rel {rel(K, ref.K.val):.2e}, dipole err {err:.2e} of {induced:.2e}")
    assert rel(K, ref.K.val) <= TOL
    dq = assert_charges(q, ref.K, st.S)
    assert err <= TOL * induced + dipole_floor(q0, st.xyz, dq)


def test_row_runs_agree_with_single_outputs(reference):
    s, _, _ = reference
    K1, tr1, _ = _run(s, 1, 1)
    for rr, rc in RUNS[1:]:
        K, tr, _ = _run(s, rr, rc)
        # same triples, contraction sums in another order: a few ulps per step
        assert rel(K, K1) <= 1e-13, (rr, rc)
        np.testing.assert_allclose(tr[:, 4], tr1[:, 4], rtol=1e-13)


def test_row_runs_fp32_products():
    """FP32 step products run the same row-run dataflow on the FP32 matrix cores."""
    s = _lattice()
    K1, _, _ = _run(s, 1, 1, precision="fp32")
    K4, _, _ = _run(s, 4, 4, precision="fp32")
    K8, _, _ = _run(s, 8, 2, precision="fp32")
    # FP32 products with FP32 accumulation in another order: agreement at FP32 rounding
    assert rel(K4, K1) <= 1e-5
    assert rel(K8, K1) <= 1e-5


def test_bad_run_length_is_refused():
    s = _cluster()
    os.environ["RTDM_RUN_REAL"] = "5"
    try:
        with pytest.raises(rtdm.RtdmError):
            gpu_context(s)
    finally:
        os.environ.pop("RTDM_RUN_REAL", None)


def test_row_runs_under_graph_capture(reference):
    """A captured step replays the row-run kernels bit for bit (the schedules
    and their runs are built when the ranges are set, never inside a capture)."""
    s, _, _ = reference
    Ke, tre, _ = _run(s, 2, 1, use_graph=0)
    Kg, trg, _ = _run(s, 2, 1, use_graph=1)
    assert np.array_equal(Ke, Kg)
    assert np.array_equal(tre[:, :6], trg[:, :6])


def test_row_runs_fp32_taylor_terms():
    """FP32-storage Taylor terms (fp32_taylor) through the FP32 row-run kernel
    agree with the single-output FP32 kernel at FP32 rounding of those terms."""
    s = _lattice()
    K1, tr1, _ = _run(s, 1, 1, precision="fp32_taylor")
    K2, tr2, _ = _run(s, 2, 1, precision="fp32_taylor")
    K8, _, _ = _run(s, 8, 1, precision="fp32_taylor")
    assert rel(K2, K1) <= 1e-9
    assert rel(K8, K1) <= 1e-9
    induced = np.abs(tr1[:, 1:4] - tr1[0, 1:4]).max()
    assert np.abs(tr2[:, 1:4] - tr1[:, 1:4]).max() <= 1e-7 * max(induced, 1e-300)


def _b4_lattice():
    return synth.diamond_lattice((3, 3, 3), 4, 10.0, 12.0, seed=33, h_model="mulliken")


def test_b4_row_runs_match_oracle_and_single_outputs():
    """b = 4 FP64 products over runs of 16 outputs of a row (RTDM_RUN_B4=16,
    the default) against the oracle and against per-output triple lists."""
    s = _b4_lattice()
    st = O.setup(s)
    ref = O.propagate(st, N_STEPS, s.dt, s.kappa, h_model=s.h_model)
    K16, tr16, _ = _run(s, 2, 2, run_b4=16)
    K1, tr1, _ = _run(s, 2, 2, run_b4=1)
    q0 = O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S)
    P0 = O.dipole(q0, st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    assert rel(K16, ref.K.val) <= TOL
    assert np.abs(tr16[:, 1:4] - ref.rows[:, 1:4]).max() <= TOL * induced + dipole_floor(q0, st.xyz)
    assert rel(K16, K1) <= 1e-13
    np.testing.assert_allclose(tr16[:, 4], tr1[:, 4], rtol=1e-13)


def test_b4_row_runs_under_graph_capture():
    s = _b4_lattice()
    Ke, tre, _ = _run(s, 2, 2, run_b4=16, use_graph=0)
    Kg, trg, _ = _run(s, 2, 2, run_b4=16, use_graph=1)
    assert np.array_equal(Ke, Kg)
    assert np.array_equal(tre[:, :6], trg[:, :6])


@pytest.mark.parametrize("precision", ["fp32_taylor", "bf16x3_taylor", "fp16x2_taylor", "fp32"])
def test_b4_row_runs_reduced_precision(precision):
    """The reduced-precision b = 4 kernel over row runs agrees with its
    per-output form at the rounding of the reduced terms (late Taylor terms
    only: 1e-8 of K; every product reduced: 1e-5)."""
    s = _b4_lattice()
    K16, _, _ = _run(s, 2, 2, run_b4=16, precision=precision)
    K1, _, _ = _run(s, 2, 2, run_b4=1, precision=precision)
    bound = 1e-5 if precision == "fp32" else 1e-8
    print(f"{precision}: runs vs per-output K rel {rel(K16, K1):.2e}")
    assert rel(K16, K1) <= bound


def test_b4_bf16_taylor_terms_from_split_storage_equal_register_split():
    """bf16x3_taylor at b = 4 over row runs takes its late Taylor terms from A
    and tau stored as BF16 hi / lo planes (k_spgemm_b4r16, the sum into U
    fused); over per-output lists the kernel splits the FP64 operands in
    registers.  The split and the products per output are the same, so the
    two agree as closely as the FP64 products over runs and over lists
    (test_b4_row_runs_match_oracle_and_single_outputs), far inside the form's
    own error (1e-8 of K against FP64)."""
    s = _b4_lattice()
    K16, tr16, q16 = _run(s, 2, 2, run_b4=16, precision="bf16x3_taylor")
    K1, tr1, q1 = _run(s, 2, 2, run_b4=1, precision="bf16x3_taylor")
    print(f"split storage vs register split: K rel {rel(K16, K1):.2e}")
    assert rel(K16, K1) <= 1e-13
    np.testing.assert_allclose(tr16[:, 4], tr1[:, 4], rtol=1e-13)
    np.testing.assert_allclose(q16, q1, rtol=0, atol=1e-13 * np.abs(q1).max())

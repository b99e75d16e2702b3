"""Reduced-precision block products against the FP64 oracle.

FP32 matrix-core products keep FP64 storage, reductions and observables.
Stated tolerances: one product within 1e-6 relative (Frobenius) of the oracle
(FP32 rounding of the operands and of each accumulation step, ~2^-24 times a
modest growth factor).  Propagation errors (dipole error relative to the
peak induced dipole, Tr(KS) relative) are printed by each test and bounded at
about 3x the measured values, so that a form that gets worse fails:
all products in FP32 lose 3.4e-2 of the kick's signal in 100 steps of the
64-atom cluster; FP32 Taylor terms from order 2 / 3 keep 1.1e-5 / 7.4e-9.

Split 16-bit forms (FP64 storage, FP32 accumulation): one product within
3e-5 relative for BF16 x3 (two 8-bit parts: the dropped lo*lo term and the
rounding of lo are each ~2^-16 of |a||b|) and within 5e-7 for FP16 x2 (two
11-bit parts, ~2^-22 each, plus FP32 accumulation).  Propagation errors are
bounded per form below at about 3x the measured values.  Every product in a
split form does not meet the 1e-6 dipole target: BF16 x3 loses the whole
induced signal (error 1.3 of its peak) and FP16 x2 4e-2 of it; only the forms
that confine the split to late Taylor terms keep the dipole error below 1e-6
(4e-8 and 3e-9 from order 3).
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import gpu_context, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("b", [4, 13])
def test_fp32_products_within_stated_tolerance(b):
    rng = np.random.default_rng(200 + b)
    xyz = synth.cluster_positions(40, rng)
    s = synth.build_system("fp32", xyz, b, 6.0, 8.0, 200 + b)
    st = O.setup(s)
    ctx = gpu_context(s, precision="fp32")
    for kind, (Cs, As, Bs, ob, pa, ca, pb, cb, pc) in {
            "AT": ("U", "A", "X", 0, st.pat_p, False, st.pat_p, False, st.pat_p),
            "UK": ("W", "U", "K", 0, st.pat_p, True, st.pat_k, True, st.pat_k),
            "WU": ("K", "W", "U", 1, st.pat_k, True, st.pat_p, True, st.pat_k)}.items():
        a = synth.random_blocks(pa.rows(), pa.col, b, 1, ca)
        bm = synth.random_blocks(pb.rows(), pb.col, b, 2, cb)
        rtdm.rtdm_upload(ctx.h, As, a)
        rtdm.rtdm_upload(ctx.h, Bs, bm)
        rtdm.rtdm_multiply(ctx.h, Cs, As, Bs, 0, ob)
        got = rtdm.rtdm_download(ctx.h, Cs, b)
        want, _ = O.spgemm(O.BSM(pa, b, a + 0j), O.BSM(pb, b, bm + 0j), pc, op_b=ob)
        e = rel(got, want.val)
        print(f"fp32 {kind} b={b}: relative error {e:.2e}")
        assert e <= 1e-6, kind
    ctx.close()


@pytest.mark.parametrize("prec,n0,bound_dip,bound_tr", [("fp32", 3, 0.1, 2e-5), ("fp32_taylor", 2, 3e-5, 4e-9),
                                                        ("fp32_taylor", 3, 2e-8, 2.5e-13)])
def test_fp32_propagation_error_stated(prec, n0, bound_dip, bound_tr):
    s = synth.config1()
    st = O.setup(s)
    ctx = gpu_context(s, precision=prec, taylor_low_from=n0)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 100)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    ref = O.propagate(st, 100, s.dt, s.kappa)
    P0 = O.dipole(O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S), st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    e_dip = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max() / induced
    e_tr = np.abs(tr[:, 4] - ref.rows[:, 4]).max() / abs(ref.rows[0, 4])
    print(f"{prec} (FP32 from Taylor order {n0}) 64-atom cluster, 100 steps: dipole error {e_dip:.2e} "
          f"of peak induced, Tr(KS) {e_tr:.2e}")
    assert e_dip <= bound_dip and e_tr <= bound_tr


@pytest.mark.parametrize("n0,bound_dip", [(2, 1e-5), (3, 8e-9)])
def test_fp32_taylor_b13_lattice_error_stated(n0, bound_dip):
    """The b = 13 FP32 step kernel (FP32 storage of the Taylor terms) on a 64-atom lattice."""
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local", h_model="mulliken")
    st = O.setup(s)
    ctx = gpu_context(s, h_model="mulliken", precision="fp32_taylor", taylor_low_from=n0)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 10)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    ref = O.propagate(st, 10, s.dt, s.kappa, h_model="mulliken")
    P0 = O.dipole(O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S), st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    e_dip = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max() / induced
    print(f"fp32_taylor (from order {n0}) b=13 lattice, 10 steps: dipole error {e_dip:.2e} of peak induced")
    assert e_dip <= bound_dip


@pytest.mark.parametrize("prec,bound", [("bf16x3", 3e-5), ("fp16x2", 5e-7)])
@pytest.mark.parametrize("b", [4, 13])
def test_split_products_within_stated_tolerance(b, prec, bound):
    rng = np.random.default_rng(300 + b)
    xyz = synth.cluster_positions(40, rng)
    s = synth.build_system("split", xyz, b, 6.0, 8.0, 300 + b)
    st = O.setup(s)
    ctx = gpu_context(s, precision=prec)
    for kind, (Cs, As, Bs, ob, pa, ca, pb, cb, pc, scale) in {
            "AT": ("U", "A", "X", 0, st.pat_p, False, st.pat_p, False, st.pat_p, 1.0),
            "AT_small": ("U", "A", "X", 0, st.pat_p, False, st.pat_p, False, st.pat_p, 1e-7),
            "UK": ("W", "U", "K", 0, st.pat_p, True, st.pat_k, True, st.pat_k, 1.0),
            "WU": ("K", "W", "U", 1, st.pat_k, True, st.pat_p, True, st.pat_k, 1.0)}.items():
        a = synth.random_blocks(pa.rows(), pa.col, b, 1, ca)
        bm = scale * synth.random_blocks(pb.rows(), pb.col, b, 2, cb)
        rtdm.rtdm_upload(ctx.h, As, a)
        rtdm.rtdm_upload(ctx.h, Bs, bm)
        rtdm.rtdm_multiply(ctx.h, Cs, As, Bs, 0, ob)
        got = rtdm.rtdm_download(ctx.h, Cs, b)
        want, _ = O.spgemm(O.BSM(pa, b, a + 0j), O.BSM(pb, b, bm + 0j), pc, op_b=ob)
        e = rel(got, want.val)
        print(f"{prec} {kind} b={b}: relative error {e:.2e}")
        assert e <= bound, kind
    ctx.close()


@pytest.mark.parametrize("prec,n0,bound_dip,bound_tr", [
    ("bf16x3", 2, 2.0, 6e-5), ("fp16x2", 2, 0.1, 2e-6),
    ("bf16x3_taylor", 2, 1.2e-3, 9e-8), ("bf16x3_taylor", 3, 1.2e-7, 1.5e-11),
    ("fp16x2_taylor", 2, 3e-5, 5e-9), ("fp16x2_taylor", 3, 9e-9, 3e-13)])
def test_split_propagation_error_stated(prec, n0, bound_dip, bound_tr):
    s = synth.config1()
    st = O.setup(s)
    ctx = gpu_context(s, precision=prec, taylor_low_from=n0)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 100)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    ref = O.propagate(st, 100, s.dt, s.kappa)
    P0 = O.dipole(O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S), st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    e_dip = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max() / induced
    e_tr = np.abs(tr[:, 4] - ref.rows[:, 4]).max() / abs(ref.rows[0, 4])
    print(f"{prec} (split from Taylor order {n0}) 64-atom cluster, 100 steps: dipole error {e_dip:.2e} "
          f"of peak induced, Tr(KS) {e_tr:.2e}")
    assert e_dip <= bound_dip and e_tr <= bound_tr


@pytest.mark.parametrize("prec,bound", [("bf16x3_taylor", 2e-8), ("fp16x2_taylor", 5e-9)])
def test_split_taylor_b13_lattice_error_stated(prec, bound):
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local", h_model="mulliken")
    st = O.setup(s)
    ctx = gpu_context(s, h_model="mulliken", precision=prec, taylor_low_from=3)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 10)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    ref = O.propagate(st, 10, s.dt, s.kappa, h_model="mulliken")
    P0 = O.dipole(O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S), st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    e_dip = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max() / induced
    print(f"{prec} (from order 3) b=13 lattice, 10 steps: dipole error {e_dip:.2e} of peak induced")
    assert e_dip <= bound


def test_fp32_step_kernels_b13_lattice_error_stated():
    """Every product of the b = 13 step on the FP32 matrix cores (operands
    rounded on load): the dipole error is of the order of the FP32 rounding
    of K relative to the small induced signal, as for the b = 4 cluster."""
    s = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=21, k0="local", h_model="mulliken")
    st = O.setup(s)
    ctx = gpu_context(s, h_model="mulliken", precision="fp32")
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    rtdm.rtdm_step(ctx.h, s.dt, 10)
    tr = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    ref = O.propagate(st, 10, s.dt, s.kappa, h_model="mulliken")
    P0 = O.dipole(O.mulliken(O.kick(st.K0, st.xyz, s.kappa), st.S), st.xyz)
    induced = np.abs(ref.rows[:, 1:4] - P0).max()
    e_dip = np.abs(tr[:, 1:4] - ref.rows[:, 1:4]).max() / induced
    e_tr = np.abs(tr[:, 4] - ref.rows[:, 4]).max() / abs(ref.rows[0, 4])
    print(f"fp32 (all products) b=13 lattice, 10 steps: dipole error {e_dip:.2e} of peak induced, Tr(KS) {e_tr:.2e}")
    assert e_dip <= 2e-2 and e_tr <= 1e-6

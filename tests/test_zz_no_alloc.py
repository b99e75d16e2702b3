"""The allocation-free product entry point (rtdm_multiply_noalloc) against
rtdm_multiply: same kernels and layouts, the b = 13 column-major operand
copies cut from the library's static device array instead of allocated.

Two contexts in a row share that array (the second with a smaller system),
each product kind must give rtdm_multiply's blocks bit for bit (and so meet
the FP64 bar against the oracle that rtdm_multiply meets in the parity
tests); a product whose copies exceed the array is refused.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, gpu_context, rel

pytestmark = pytest.mark.gpu

KINDS = {
    # kind: (C slot, A slot, B slot, op_b, A complex, B complex, alpha)
    "XH": ("A", "X", "H", 0, False, False, 1.0),
    "AT": ("U", "A", "X", 0, False, False, 0.37),
    "UK": ("W", "U", "K", 0, True, True, 1.0),
    "WU": ("K", "W", "U", 1, True, True, 1.0),
}


def _pattern(ctx, slot, n):
    rp, col = rtdm.rtdm_pattern(ctx.h, slot)
    return O.Pattern(n, 0.0, rp, col)


def _check_kinds(s, seed):
    ctx = gpu_context(s)
    try:
        for kind, (Cs, As, Bs, ob, ca, cb, alpha) in KINDS.items():
            pa, pb, pc = _pattern(ctx, As, s.n_atoms), _pattern(ctx, Bs, s.n_atoms), _pattern(ctx, Cs, s.n_atoms)
            a = synth.random_blocks(pa.rows(), pa.col, s.b, seed, ca)
            bm = synth.random_blocks(pb.rows(), pb.col, s.b, seed + 1, cb)
            rtdm.rtdm_upload(ctx.h, As, a)
            rtdm.rtdm_upload(ctx.h, Bs, bm)
            rtdm.rtdm_multiply(ctx.h, Cs, As, Bs, 0, ob, alpha)
            want = rtdm.rtdm_download(ctx.h, Cs, s.b)
            rtdm.rtdm_upload(ctx.h, Cs, np.zeros_like(want))
            rtdm.rtdm_multiply_noalloc(ctx.h, Cs, As, Bs, 0, ob, alpha)
            got = rtdm.rtdm_download(ctx.h, Cs, s.b)
            print(f"{s.name} {kind}: noalloc vs multiply max |diff| {np.abs(got - want).max():.1e}")
            assert np.array_equal(got, want), kind
            ref, _ = O.spgemm(O.BSM(pa, s.b, a + 0j), O.BSM(pb, s.b, bm + 0j), pc, alpha=alpha, op_b=ob)
            assert rel(got, ref.val) <= TOL, kind
    finally:
        ctx.close()


def test_noalloc_multiply_equals_multiply_on_two_systems_in_a_row():
    big = synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=27, k0="local", h_model="mulliken")
    rng = np.random.default_rng(28)
    small = synth.build_system("cl23_b13", synth.cluster_positions(23, rng), 13, 6.0, 8.0, 28)
    _check_kinds(big, 31)
    _check_kinds(small, 41)          # the second call, with a smaller input, reuses the same array
    _check_kinds(synth.config1(), 51)  # b = 4: no copies, the plain product kernels


def test_noalloc_multiply_refuses_operands_beyond_the_array():
    s = synth.diamond_lattice((3, 3, 3), 13, 10.0, 16.0, seed=29, k0="local", h_model="mulliken")
    ctx = gpu_context(s)
    try:
        nnzb = rtdm.rtdm_pattern(ctx.h, "K")[1].size
        need = 4 * nnzb * 13 * 13 * 8            # W U^dagger: two planes of W and two of U, column-major
        assert need > (128 << 20)
        with pytest.raises(rtdm.RtdmError) as e:
            rtdm.rtdm_multiply_noalloc(ctx.h, "K", "W", "U", 0, 1, 1.0)
        assert e.value.code == -1              # RTDM_E_ARG
        rtdm.rtdm_multiply_noalloc(ctx.h, "A", "X", "H", 0, 0, 1.0)   # one real plane fits
    finally:
        ctx.close()

"""Full-size checks on the benchmark workload (4,096-atom lattice, b = 13).

Products run through the same entry points and launch configuration as the
timed steps; the oracle recomputes sampled output rows one by one (rows at the
start, the middle and the end of the atom order, so surface and bulk atoms
are both covered).  The propagation itself is checked through properties that
hold at any size: exact Hermiticity after each step, conservation of Tr(KS)
to the size of the Taylor and truncation defects, and a small unitarity error.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth
from tests._common import TOL, gpu_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    s = synth.config2()
    st = O.setup(s)
    ctx = gpu_context(s, h_model="mulliken")
    yield s, st, ctx
    ctx.close()


def _sample_rows(n):
    return [(0, 3), (n // 2 - 2, n // 2 + 1), (n - 3, n)]


@pytest.mark.parametrize("kind", ["XH", "AT", "UK", "WU"])
def test_fullsize_product_sampled_rows(big, kind):
    s, st, ctx = big
    b, h = s.b, ctx.h
    pp, ph, pk = st.pat_p, st.pat_hs, st.pat_k
    spec = {"XH": ("A", "X", "H", 0, (pp, False), (ph, False), pp, 1.0),
            "AT": ("U", "A", "X", 0, (pp, False), (pp, False), pp, 0.05 / 3),
            "UK": ("W", "U", "K", 0, (pp, True), (pk, True), pk, 1.0),
            "WU": ("K", "W", "U", 1, (pk, True), (pp, True), pk, 1.0)}[kind]
    Cs, As, Bs, ob, (pa, ca), (pb, cb), pc, alpha = spec
    a = synth.random_blocks(pa.rows(), pa.col, b, 31, ca)
    bm = synth.random_blocks(pb.rows(), pb.col, b, 32, cb)
    rtdm.rtdm_upload(h, As, a)
    rtdm.rtdm_upload(h, Bs, bm)
    rtdm.rtdm_multiply(h, Cs, As, Bs, 0, ob, alpha)
    got = rtdm.rtdm_download(h, Cs, b)
    A = O.BSM(pa, b, a.astype(np.complex128))
    B = O.BSM(pb, b, bm.astype(np.complex128))
    del a, bm
    r = pc.rows()
    for lo, hi in _sample_rows(s.n_atoms):
        want, _ = O.spgemm(A, B, pc, alpha=alpha, op_b=ob, rows=(lo, hi))
        sel = (r >= lo) & (r < hi)
        g, w = got[sel], want.val[sel]
        assert np.linalg.norm(g - w) <= TOL * np.linalg.norm(w), (kind, lo)
        assert np.abs(g - w).max() <= TOL * np.abs(w).max(), (kind, lo)


def test_fullsize_triple_counts(big):
    s, st, ctx = big
    out = {k: rtdm.rtdm_schedule_stats(ctx.h, k) for k in ("XH", "AT", "UK", "WU")}
    # the pattern of every output: one output block per kept pair
    assert out["XH"][0] == st.pat_p.nnzb and out["UK"][0] == st.pat_k.nnzb
    # per-row triple counts of the AT product on the sampled rows, by brute force
    pp = st.pat_p
    rows = [set(pp.col[pp.row_ptr[i]:pp.row_ptr[i + 1]].tolist()) for i in range(s.n_atoms)]
    for i in (0, s.n_atoms // 2, s.n_atoms - 1):
        cnt = sum(len(rows[i] & rows[j]) for j in rows[i])
        Z = O.zeros(pp, s.b)
        _, t = O.spgemm(Z, Z, pp, rows=(i, i + 1))
        assert t == cnt
    # expected size (a sampled count of the lattice's triples): about 1.06e8 triples for A T on this lattice
    assert 0.9e8 < out["AT"][1] < 1.2e8


def test_fullsize_steps_keep_invariants(big):
    s, st, ctx = big
    h = ctx.h
    ctx.load_system(s)
    it, res = rtdm.rtdm_build_inverse(h)
    assert it <= 10 and res <= 1e-10
    rtdm.rtdm_apply_kick(h, s.kappa)
    obs0 = rtdm.rtdm_observables(h)
    rtdm.rtdm_step(h, s.dt, 3)
    tr = rtdm.rtdm_dipole_trace(h)
    assert tr.shape == (3, 7) and np.all(np.isfinite(tr[:, :6]))
    # Tr(KS) is conserved to the truncation / Taylor defect
    assert np.abs(tr[:, 4] - obs0[3]).max() <= 1e-6 * abs(obs0[3])
    # the propagator is unitary in the S metric to the same level
    u = rtdm.rtdm_unitarity(h)
    assert u[0] < 1e-5
    # K is exactly Hermitian after every step
    K = rtdm.rtdm_download(h, "K", s.b)
    t = st.pat_k.transpose_index()
    assert np.array_equal(K, np.conj(np.transpose(K[t], (0, 2, 1))))

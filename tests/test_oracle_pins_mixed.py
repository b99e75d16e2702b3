"""Pins of the oracle for atoms with different numbers of functions (oracle/mixed.py).

* Equal sizes: the dense masked form equals oracle.py's block-sparse form
  (a separate implementation: Gustavson products in C over block storage).
* Mixed sizes: the dense form equals oracle.py run on the same system with
  every atom padded to 13 functions (identity in S on the padded functions,
  zeros in H0 and K0), which is the reduction the GPU library relies on; the
  padded functions must stay decoupled for the two to agree.
* No truncation (ranges wider than the cluster): the Hotelling inverse is
  LAPACK's inverse, the propagator is the Taylor polynomial of
  -i dt S^-1 H written out densely, and K after n fixed-H steps is
  U^n K0 U^dagger^n.
"""

import numpy as np
import pytest

from oracle import mixed as M
from oracle import oracle as O
from paper_1404_5776_amd import synth
from tests._common import padded_system as _padded, strip_padding as _strip

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _as_mixed(sys_):
    """An equal-size system in the mixed representation."""
    def conv(c):
        return synth.MixedCOO(c.rows, c.cols, c.data.reshape(-1))
    return synth.MixedSystem(name=sys_.name, xyz=sys_.xyz, nbf=sys_.nbf, R_HS=sys_.R_HS, R_K=sys_.R_K,
                             R_P=sys_.R_P, S=conv(sys_.S), H0=conv(sys_.H0), K0=conv(sys_.K0))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("h_model", ["fixed", "mulliken"])
def test_equal_sizes_match_the_block_sparse_oracle(h_model):
    s = synth.random_cluster(40, 4, 8.0, 12.0, 61, k0="exact")
    st = O.setup(s)
    ref = O.propagate(st, 6, 0.05, (0.01, 0.0, 0.0), h_model=h_model)
    ms = _as_mixed(s)
    mt = M.setup(ms)
    got = M.propagate(mt, 6, 0.05, (0.01, 0.0, 0.0), h_model=h_model)
    Kd = _strip(ref.K, ms)
    assert _rel(got.K, Kd) < 1e-12
    induced = np.abs(ref.rows[:, 1:4] - ref.rows[0, 1:4]).max()
    assert np.abs(got.rows[:, 1:4] - ref.rows[:, 1:4]).max() < 1e-9 * induced
    assert np.abs(got.rows[:, 4] - ref.rows[:, 4]).max() < 1e-12 * abs(ref.rows[0, 4])
    assert got.inverse_iters == ref.inverse.iters


@pytest.mark.parametrize("h_model", ["fixed", "mulliken"])
def test_mixed_sizes_match_the_padded_block_sparse_oracle(h_model):
    ms = synth.mixed_cluster(36, 5, h_model=h_model)
    assert set(ms.nbf.tolist()) == {4, 13}
    mt = M.setup(ms)
    got = M.propagate(mt, 5, 0.05, (0.01, 0.0, 0.0), h_model=h_model, inv_tol=1e-12)
    ps = _padded(ms)
    st = O.setup(ps)
    ref = O.propagate(st, 5, 0.05, (0.01, 0.0, 0.0), h_model=h_model, inv_tol=1e-12)
    assert _rel(got.K, _strip(ref.K, ms)) < 1e-11
    # the padded functions of K stay exactly zero
    r = ref.K.pat.rows()
    for p in range(ref.K.pat.nnzb):
        i, j = int(r[p]), int(ref.K.pat.col[p])
        blk = ref.K.val[p].copy()
        blk[:ms.nbf[i], :ms.nbf[j]] = 0.0
        assert not blk.any()
    induced = np.abs(ref.rows[:, 1:4] - ref.rows[0, 1:4]).max()
    assert np.abs(got.rows[:, 1:4] - ref.rows[:, 1:4]).max() < 1e-9 * induced
    assert np.abs(got.rows[:, 4] - ref.rows[:, 4]).max() < 1e-12 * abs(ref.rows[0, 4])


def test_untruncated_mixed_propagation_is_the_dense_taylor_polynomial():
    ms = synth.mixed_cluster(16, 9, R_HS=60.0, R_K=60.0)      # every pair kept
    mt = M.setup(ms)
    assert mt.mask_k.all() and mt.mask_hs.all()
    dt, n, p = 0.05, 4, 5
    got = M.propagate(mt, n, dt, (0.02, -0.01, 0.0), inv_tol=1e-14)
    Sinv = np.linalg.inv(mt.S)
    assert _rel(got.X, Sinv) < 1e-12
    A = Sinv @ mt.H0
    G = -1j * dt * A
    U = np.zeros_like(G)
    term = np.eye(G.shape[0], dtype=complex)
    fact = 1.0
    for k in range(p + 1):
        U = U + term / fact
        term = term @ G
        fact *= k + 1
    assert _rel(got.U, U) < 1e-12
    K = M.kick(mt, mt.K0, (0.02, -0.01, 0.0))
    for _ in range(n):
        K = U @ K @ U.conj().T
    assert _rel(got.K, K) < 1e-11
    # Mulliken charges sum to Re tr(K S)
    assert abs(got.q.sum() - np.trace(got.K @ mt.S).real) < 1e-11 * abs(got.q.sum())

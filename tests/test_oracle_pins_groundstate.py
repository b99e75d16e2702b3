"""Pins of the oracle's ground state by truncated trace-correcting purification.

Independent references: scipy's generalized eigendecomposition (the exact
occupied projector), the defining properties of a ground-state density
matrix (K S K = K, Tr(K S) = n_occ, symmetry), and dense eigenvalues for the
Gershgorin bounds.
"""

import numpy as np
import pytest
from scipy.linalg import eigh

from oracle import oracle as O
from paper_1404_5776_amd import synth


def _sys(cells=(2, 2, 2), b=4, R_HS=10.0, R=40.0, seed=5):
    s = synth.diamond_lattice(cells, b, R_HS, R, seed=seed, k0="exact")
    st = O.setup(s)
    X = O.hotelling(st.S, st.pat_p, tol=1e-14).X
    return s, st, X


def test_gershgorin_bounds_contain_the_spectrum():
    s, st, X = _sys()
    A, _ = O.spgemm(X, st.H0, st.pat_p)
    lo, hi = O.gershgorin(A)
    ev = eigh(st.H0.to_dense().real, st.S.to_dense().real, eigvals_only=True)
    assert lo <= ev.min() and ev.max() <= hi
    assert hi - lo < 10 * (ev.max() - ev.min())       # not absurdly loose


@pytest.mark.parametrize("b", [4, 13])
def test_untruncated_purification_is_the_occupied_projector(b):
    s, st, X = _sys(b=b, R_HS=10.0, R=40.0)
    n_occ = synth.n_occupied(s.n_atoms, b)
    gs = O.ground_state(st.S, st.H0, X, st.pat_p, st.pat_k, n_occ)
    Sd, Hd = st.S.to_dense().real, st.H0.to_dense().real
    w, V = eigh(Hd, Sd)
    Kref = V[:, :n_occ] @ V[:, :n_occ].T
    K = gs.K.to_dense().real
    print(f"b={b}: {gs.iters} iterations, idempotency {gs.idempotency[-1]:.2e}, "
          f"gap {w[n_occ] - w[n_occ - 1]:.3f}")
    assert np.abs(K - Kref).max() < 1e-8 * np.abs(Kref).max()
    assert abs(np.trace(K @ Sd) - n_occ) < 1e-8 * n_occ
    assert np.abs(K @ Sd @ K - K).max() < 1e-8 * np.abs(K).max()
    assert np.array_equal(K, K.T)


def test_truncated_purification_keeps_trace_and_symmetry():
    s = synth.diamond_lattice((3, 3, 3), 4, 10.0, 8.0, seed=6, k0="local")
    st = O.setup(s)
    X = O.hotelling(st.S, st.pat_p).X
    n_occ = synth.n_occupied(s.n_atoms, 4)
    gs = O.ground_state(st.S, st.H0, X, st.pat_p, st.pat_k, n_occ)
    K = gs.K
    assert np.array_equal(K.val, K.conj_transpose().val)
    tr = O.mulliken(K, st.S).sum()
    print(f"truncated: {gs.iters} iterations, idempotency {gs.idempotency[-1]:.2e}, Tr(KS) {tr:.8f} of {n_occ}")
    assert abs(tr - n_occ) < 1e-3 * n_occ
    # close to the exact ground state restricted to the range, as the range grows
    Sd, Hd = st.S.to_dense().real, st.H0.to_dense().real
    w, V = eigh(Hd, Sd)
    Kref = V[:, :n_occ] @ V[:, :n_occ].T
    errs = []
    for R in (8.0, 12.0, 16.0):
        pat = O.pattern(s.xyz, R)
        Xr = O.hotelling(st.S, pat).X
        g = O.ground_state(st.S, st.H0, Xr, pat, pat, n_occ)
        mask = np.zeros_like(Kref, dtype=bool)
        for i, j in zip(pat.rows(), pat.col):
            mask[4 * i:4 * i + 4, 4 * j:4 * j + 4] = True
        errs.append(np.abs(g.K.to_dense().real - Kref)[mask].max())
    print("max error on the kept blocks vs range 8/12/16:", errs)
    assert errs[0] > errs[1] > errs[2]


def test_branch_rule_and_iteration_count_recorded():
    s, st, X = _sys(b=4)
    n_occ = synth.n_occupied(s.n_atoms, 4)
    gs = O.ground_state(st.S, st.H0, X, st.pat_p, st.pat_k, n_occ)
    assert gs.iters == len(gs.idempotency) and gs.iters >= 5
    assert gs.branches < (1 << gs.iters)
    assert gs.idempotency[-1] <= 1e-10 * n_occ

"""Oracle for atoms with different numbers of support functions (Sec. III:
each element has its own basis size, e.g. SZP and SZ2P in Sec. V).

TEST INFRASTRUCTURE ONLY, like oracle.py: the tests use it to check the GPU
library; nothing on the product path imports it.

Plain FP64 over dense matrices indexed by support function (the functions of
atom i are rows off[i] .. off[i+1]-1).  A cut-off is a mask over function
pairs built from the atom-pair rule of oracle.py (kept iff i == j or
|r_i - r_j|^2 < R^2), and every truncated product is the dense product with
the output mask applied, P_C(A B) = mask_C * (A @ B): operands that already
vanish outside their own range give the same sum over k as the block form.
The method is oracle.py's, step for step and with the same readings (Taylor
order 5 recursion, truncation points, Hotelling stopping rule, Mulliken
charges over the pairs kept in both K and S, midpoint charges extrapolated
from the last two steps, on-site shift on each of the atom's own functions,
kick phases, dipole about the centroid); only the storage differs.  Scope:
the exponential-midpoint step with a fixed or Mulliken H, block-Jacobi start.
"""

from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

from oracle import oracle as O


@dataclasses.dataclass
class MixedSetup:
    xyz: np.ndarray
    nbf: np.ndarray
    off: np.ndarray            # function offset of each atom (n + 1)
    atom: np.ndarray           # atom of each function
    mask_hs: np.ndarray        # (nf, nf) bool
    mask_p: np.ndarray
    mask_k: np.ndarray
    S: np.ndarray              # dense, masked to R_HS
    H0: np.ndarray
    K0: np.ndarray             # masked to R_K


def atom_mask(xyz: np.ndarray, R: float) -> np.ndarray:
    """(n, n) atom pairs kept at range R (the rule of oracle.pattern)."""
    d = xyz[:, None, :] - xyz[None, :, :]
    d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
    return (d2 < R * R) | np.eye(xyz.shape[0], dtype=bool)


def function_mask(am: np.ndarray, atom: np.ndarray) -> np.ndarray:
    return am[np.ix_(atom, atom)]


def from_blocks(coo, off: np.ndarray, nf: int) -> np.ndarray:
    """Dense matrix from concatenated row-major blocks of per-atom sizes."""
    out = np.zeros((nf, nf), dtype=np.result_type(coo.data, np.float64))
    at = 0
    for i, j in zip(coo.rows, coo.cols):
        ni, nj = off[i + 1] - off[i], off[j + 1] - off[j]
        out[off[i]:off[i + 1], off[j]:off[j + 1]] = coo.data[at:at + ni * nj].reshape(ni, nj)
        at += ni * nj
    return out


def to_blocks(M: np.ndarray, off: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Blocks (i, j) of a dense matrix, row-major, concatenated in the given order."""
    return np.concatenate([M[off[i]:off[i + 1], off[j]:off[j + 1]].ravel() for i, j in zip(rows, cols)])


def setup(sys_) -> MixedSetup:
    nbf = np.asarray(sys_.nbf, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(nbf)])
    nf = int(off[-1])
    atom = np.repeat(np.arange(nbf.size), nbf)
    m_hs = function_mask(atom_mask(sys_.xyz, sys_.R_HS), atom)
    m_p = function_mask(atom_mask(sys_.xyz, sys_.R_P), atom)
    m_k = function_mask(atom_mask(sys_.xyz, sys_.R_K), atom)
    S = from_blocks(sys_.S, off, nf) * m_hs
    H0 = from_blocks(sys_.H0, off, nf) * m_hs
    K0 = from_blocks(sys_.K0, off, nf) * m_k
    return MixedSetup(sys_.xyz, nbf, off, atom, m_hs, m_p, m_k, S, H0, K0)


def product(A: np.ndarray, B: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """P_C(A B): the product with the output range applied."""
    return (A @ B) * mask


def frob(M: np.ndarray) -> float:
    return float(np.sqrt(np.sum(np.abs(M) ** 2)))


def block_jacobi_start(st: MixedSetup) -> np.ndarray:
    """X_0 = blockdiag(S_ii^-1)."""
    X = np.zeros_like(st.S)
    for i in range(st.nbf.size):
        a, b = st.off[i], st.off[i + 1]
        X[a:b, a:b] = np.linalg.inv(st.S[a:b, a:b])
    return X


def hotelling(st: MixedSetup, tol: float = 1e-10, max_iter: int = 50):
    """X_{k+1} = P_P(2 X_k - P_P(X_k P_P(S X_k))) from the block-Jacobi start,
    residual ||X_{k+1} - X_k||_F / ||X_{k+1}||_F (Sec. V.A)."""
    X = block_jacobi_start(st)
    res: List[float] = []
    for k in range(max_iter):
        W = product(st.S, X, st.mask_p)
        XW = product(X, W, st.mask_p)
        Xn = 2.0 * X - XW
        r = frob(Xn - X) / frob(Xn)
        res.append(r)
        if not np.isfinite(r) or (k >= 1 and r > res[-2]):
            raise RuntimeError(f"Hotelling iteration diverged: {res[-3:]}")
        X = Xn
        if r <= tol:
            return X, res
    raise RuntimeError(f"Hotelling iteration did not converge: {res[-3:]}")


def taylor_propagator(A: np.ndarray, dt: float, p: int, mask_u: np.ndarray) -> np.ndarray:
    """U = sum_{n=0}^{p} T_n, T_0 = I, T_1 = -i dt A, T_n = P_U((-i dt / n) A T_{n-1})."""
    T = np.eye(A.shape[0], dtype=np.complex128)
    U = T.copy()
    if p >= 1:
        T = -1j * dt * A
        U = U + T
    for n in range(2, p + 1):
        T = ((-1j * dt / n) * (A @ T)) * mask_u
        U = U + T
    return U


def mulliken(st: MixedSetup, K: np.ndarray) -> np.ndarray:
    """q_i = Re sum over atom i's functions mu of sum_nu K_mu,nu S_nu,mu, pairs
    kept in both K and S."""
    per_fn = np.sum((K * st.mask_k * st.mask_hs) * st.S.T, axis=1).real
    return np.bincount(st.atom, weights=per_fn, minlength=st.nbf.size)


def kick(st: MixedSetup, K: np.ndarray, kappa: Sequence[float]) -> np.ndarray:
    """K_mu,nu <- exp(i kappa . (r_a(mu) - r_a(nu))) K_mu,nu."""
    ph = st.xyz[st.atom] @ np.asarray(kappa, dtype=np.float64)
    return K * np.exp(1j * (ph[:, None] - ph[None, :]))


def hamiltonian(st: MixedSetup, q_eff, q_ref, h_model: str, h_gain: float) -> np.ndarray:
    """H0, plus g (q_eff,i - q_ref,i) on the diagonal of atom i's own functions."""
    if h_model == "fixed":
        return st.H0
    return st.H0 + np.diag(h_gain * (q_eff - q_ref)[st.atom])


@dataclasses.dataclass
class Trace:
    rows: np.ndarray           # (n_steps, 6): t, Px, Py, Pz, Tr(KS), herm_err
    K: np.ndarray
    U: np.ndarray
    X: np.ndarray
    q: np.ndarray
    inverse_iters: int


def propagate(st: MixedSetup, n_steps: int, dt: float, kappa: Sequence[float], h_model: str = "fixed",
              h_gain: float = 0.5, p: int = 5, inv_tol: float = 1e-10) -> Trace:
    """Kick K0 and take n exponential-midpoint steps (Secs. II.A, II.B, IV, V.A)."""
    X, res = hotelling(st, tol=inv_tol)
    q_ref = mulliken(st, st.K0)
    K = kick(st, st.K0, kappa)
    q_cur = mulliken(st, K)
    q_prev = q_cur.copy()
    U = None
    rows = []
    for s in range(n_steps):
        if h_model == "mulliken" or U is None:
            H = hamiltonian(st, q_cur + 0.5 * (q_cur - q_prev), q_ref, h_model, h_gain)
            A = product(X, H, st.mask_p)
            U = taylor_propagator(A, dt, p, st.mask_p)
        W = product(U, K, st.mask_k)
        Kn = product(W, U.conj().T, st.mask_k)
        he = frob(Kn - Kn.conj().T) / frob(Kn)
        K = 0.5 * (Kn + Kn.conj().T)
        q_prev, q_cur = q_cur, mulliken(st, K)
        P = O.dipole(q_cur, st.xyz)
        rows.append([(s + 1) * dt, P[0], P[1], P[2], q_cur.sum(), he])
    return Trace(np.asarray(rows).reshape(-1, 6), K, U, X, q_cur, len(res))

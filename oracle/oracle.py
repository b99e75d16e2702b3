"""Oracle for the truncated block-sparse propagation step (O'Rourke & Bowler, arXiv:1404.5776).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it to check the GPU library.  Nothing on the product
path imports it, and it imports nothing from the product path (only the seeded
input generator, which holds none of the method's arithmetic).

Plain FP64 (complex128) throughout.  The only compiled piece is oracle.c (the
cut-off pattern and the masked block product); everything else is numpy over
the oracle's own block storage, written in the order the paper gives:

* Sec. II.A  density matrix rho = phi K phi over non-orthogonal support
  functions with overlap S; all matrices vanish beyond a spatial cut-off.
* Sec. II.A  Liouville equation i dK/dt = S^-1 H K - K H S^-1, solved by
  K(t) = U K(t0) U^dagger with U a product of short-time propagators
  U(t+dt, t) = exp(-i S^-1 H dt) (Eq. prop), the exponential evaluated by a
  truncated Taylor series (Eq. matrix_exp) and H taken at the midpoint
  t + dt/2 (exponential midpoint, Eq. EM).
* Sec. IV.B  six terms of the Taylor expansion.
* Sec. V.A   S^-1 from Hotelling's method, computed once (atoms fixed);
  S^-1 and S^-1 H both truncated.
* Sec. II.B  induced dipole from the density; Sec. IV charge Tr(KS) and
  unitarity of the propagator with respect to the non-orthogonal basis.

Where the paper is silent the readings are (each listed in the design notes):

1. Taylor order p = 5: orders 0..5, "six terms".
2. T_0 = I, T_1 = -i dt A, T_n = P_U((-i dt / n) A T_{n-1}) for n >= 2,
   U = sum_n T_n; the scalar multiplies the product before truncation.
3. R_X = R_A = R_U = max(R_K, R_HS); the intermediate W = U K lives on K's range.
4. (i,j) kept iff i == j or dx*dx+dy*dy+dz*dz < R*R in float64.
5. Unitarity measured as ||P_P(U^dagger P_P(S U)) - S||_F / ||S||_F.
6. K' = P_K(P_K(U K) U^dagger) is Hermitised, K <- (K' + K'^dagger)/2, every step.
7. Hotelling X_{k+1} = P_X(2 X_k - X_k P_X(S X_k)), residual
   ||X_{k+1} - X_k||_F / ||X_{k+1}||_F, stop at tol; divergence (residual
   rising after the first iteration, or non-finite) falls back to the
   block-Jacobi start.
8. Midpoint H from linearly extrapolated Mulliken charges
   q_mid = 1.5 q(t) - 0.5 q(t - dt), q(-dt) := q(0+).
9. H = H0 + g diag(q_mid - q_ref) on every diagonal element of atom i's
   diagonal block, q_i = Re sum_j tr(K_ij S_ji), q_ref = q(K0) before the kick.
10. Kick K_ij <- exp(i kappa . (r_i - r_j)) K_ij.
11. Dipole P = -sum_i (r_i - r_c) q_i with r_c the centroid of the atoms.
12. ETRS: each half-step exponential is its own truncated Taylor series and
    their product is truncated to P_U; M4: the commutator is the difference
    of the two truncated products, exp(M) the complex recursion
    T_n = P_U(M T_{n-1}) / n.
13. Charges at a time point t + theta dt: extrapolated from q(t - dt), q(t);
    in corrector passes interpolated between q(t) and the q(t + dt) of the
    previous pass.
14. Field: the electrons carry the energy +E(t).(r - r_c) in the position
    model <i|r|j> = (r_i + r_j)/2 S_ij; a kick exp(i kappa.r) is then the
    impulsive field of integral -kappa.
15. Spectrum: rectangle-rule damped transform over the recorded steps,
    alpha_jj = F[P_j - P_j(0)] / F[E_j], F[E] = -kappa for a kick.
16. Ground state: trace-correcting purification of P(S^-1 H) from Gershgorin
    bounds, K = (P_K(Z S^-1) + transpose) / 2.
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_oracle() -> str:
    """Compile oracle.c with gcc (plain C, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", src, "-o", _SO + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_oracle()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_pattern_count.argtypes = [i64, P, ctypes.c_double, P]
        L.oracle_pattern_fill.argtypes = [i64, P, ctypes.c_double, P, P]
        L.oracle_spgemm.argtypes = [i64, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, ctypes.c_int,
                                    P, P, P, ctypes.c_double, ctypes.c_double, i64, i64]
        L.oracle_spgemm.restype = i64
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """OpenMP threads of the compiled oracle (0: keep); returns the count in force."""
    return int(lib().oracle_set_threads(int(n)))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# storage
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Pattern:
    """Cut-off pattern of one range (Sec. II.A): CSR of kept atom pairs."""

    n: int
    R: float
    row_ptr: np.ndarray  # int64 (n+1)
    col: np.ndarray      # int32 (nnzb)

    @property
    def nnzb(self) -> int:
        return int(self.col.size)

    def rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def index(self, i, j) -> np.ndarray:
        """Positions of blocks (i, j) (arrays), -1 where absent."""
        i = np.asarray(i, dtype=np.int64)
        j = np.asarray(j, dtype=np.int64)
        key = self.rows() * self.n + self.col
        q = i * self.n + j
        pos = np.searchsorted(key, q)
        pos = np.minimum(pos, key.size - 1)
        return np.where(key[pos] == q, pos, -1)

    def transpose_index(self) -> np.ndarray:
        """t[p] = position of (j, i) for the block p = (i, j)."""
        t = self.index(self.col, self.rows())
        assert np.all(t >= 0), "cut-off patterns are symmetric"
        return t


def pattern(xyz: np.ndarray, R: float) -> Pattern:
    """Kept pairs of the spatial cut-off R (Sec. II.A), brute force in oracle.c."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    n = xyz.shape[0]
    cnt = np.zeros(n, dtype=np.int64)
    lib().oracle_pattern_count(n, _ptr(xyz), float(R), _ptr(cnt))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=row_ptr[1:])
    col = np.zeros(int(row_ptr[-1]), dtype=np.int32)
    lib().oracle_pattern_fill(n, _ptr(xyz), float(R), _ptr(row_ptr), _ptr(col))
    return Pattern(n, float(R), row_ptr, col)


@dataclasses.dataclass
class BSM:
    """Atom-pair blocked matrix on a cut-off pattern, complex128 blocks."""

    pat: Pattern
    b: int
    val: np.ndarray  # (nnzb, b, b) complex128

    def copy(self) -> "BSM":
        return BSM(self.pat, self.b, self.val.copy())

    def conj_transpose(self) -> "BSM":
        t = self.pat.transpose_index()
        return BSM(self.pat, self.b, np.conj(np.transpose(self.val[t], (0, 2, 1))))

    def to_dense(self) -> np.ndarray:
        n, b = self.pat.n, self.b
        out = np.zeros((n * b, n * b), dtype=np.complex128)
        r = self.pat.rows()
        for p in range(self.pat.nnzb):
            i, j = int(r[p]), int(self.pat.col[p])
            out[i * b:(i + 1) * b, j * b:(j + 1) * b] = self.val[p]
        return out


def zeros(pat: Pattern, b: int) -> BSM:
    return BSM(pat, b, np.zeros((pat.nnzb, b, b), dtype=np.complex128))


def identity(pat: Pattern, b: int) -> BSM:
    m = zeros(pat, b)
    d = pat.index(np.arange(pat.n), np.arange(pat.n))
    m.val[d] = np.eye(b)
    return m


def from_coo(coo, pat: Pattern, b: int) -> BSM:
    """Place generator blocks on a pattern; blocks outside the pattern are dropped."""
    m = zeros(pat, b)
    pos = pat.index(coo.rows, coo.cols)
    keep = pos >= 0
    m.val[pos[keep]] = coo.data[keep]
    return m


def frob(m: BSM) -> float:
    return float(np.sqrt(np.sum(np.abs(m.val) ** 2)))


def axpby(a: complex, x: BSM, c: complex, y: BSM) -> BSM:
    assert x.pat is y.pat
    return BSM(x.pat, x.b, a * x.val + c * y.val)


# ----------------------------------------------------------------------------
# the truncated product
# ----------------------------------------------------------------------------

def spgemm(A: BSM, B: BSM, pat_c: Pattern, alpha: complex = 1.0, op_a: int = 0, op_b: int = 0,
           rows: Optional[Tuple[int, int]] = None) -> Tuple[BSM, int]:
    """C = P_C(alpha op(A) op(B)) (op: 0 identity, 1 conjugate transpose).

    Returns C and the number of contributing (i, k, j) block triples.  With
    ``rows`` only those output rows are computed (the others stay zero).
    """
    b = A.b
    n = A.pat.n
    # the C product reads interleaved complex128 blocks: real arrays are converted
    a_val = np.ascontiguousarray(A.val, dtype=np.complex128).view(np.float64)
    b_val = np.ascontiguousarray(B.val, dtype=np.complex128).view(np.float64)
    C = zeros(pat_c, b)
    c_val = C.val.view(np.float64)
    lo, hi = (0, n) if rows is None else rows
    t = lib().oracle_spgemm(n, b, _ptr(A.pat.row_ptr), _ptr(A.pat.col), _ptr(a_val), int(op_a),
                            _ptr(B.pat.row_ptr), _ptr(B.pat.col), _ptr(b_val), int(op_b),
                            _ptr(pat_c.row_ptr), _ptr(pat_c.col), _ptr(c_val),
                            float(np.real(alpha)), float(np.imag(alpha)), int(lo), int(hi))
    return C, int(t)


# ----------------------------------------------------------------------------
# the method
# ----------------------------------------------------------------------------

def block_jacobi_start(S: BSM, pat_x: Pattern) -> BSM:
    """X_0 = blockdiag(S_ii^-1) (warm start of the inverse iteration)."""
    X = zeros(pat_x, S.b)
    ds = S.pat.index(np.arange(S.pat.n), np.arange(S.pat.n))
    dx = pat_x.index(np.arange(pat_x.n), np.arange(pat_x.n))
    X.val[dx] = np.linalg.inv(S.val[ds])
    return X


def cold_start(S: BSM, pat_x: Pattern) -> BSM:
    """X_0 = I / lambda_ub with lambda_ub the largest absolute row sum of S."""
    n, b = S.pat.n, S.b
    rowsum = np.zeros(n * b)
    r = S.pat.rows()
    absrow = np.abs(S.val).sum(axis=2)          # (nnzb, b)
    np.add.at(rowsum.reshape(n, b), r, absrow)
    lam = rowsum.max()
    X = identity(pat_x, b)
    X.val /= lam
    return X


@dataclasses.dataclass
class InverseResult:
    X: BSM
    iters: int
    residuals: List[float]
    fell_back: bool = False


def hotelling(S: BSM, pat_x: Pattern, X0: Optional[BSM] = None, tol: float = 1e-10,
              max_iter: int = 50) -> InverseResult:
    """Truncated Hotelling inverse of S (Sec. V.A), X_{k+1} = P_X(2 X_k - X_k P_X(S X_k))."""

    def run(X):
        res: List[float] = []
        for k in range(max_iter):
            W, _ = spgemm(S, X, pat_x)
            XW, _ = spgemm(X, W, pat_x)
            Xn = axpby(2.0, X, -1.0, XW)
            d = axpby(1.0, Xn, -1.0, X)
            r = frob(d) / frob(Xn)
            res.append(r)
            if not np.isfinite(r) or (k >= 1 and r > res[-2]):
                return Xn, res, False
            X = Xn
            if r <= tol:
                return X, res, True
        return X, res, False

    fell_back = False
    start = X0 if X0 is not None else block_jacobi_start(S, pat_x)
    X, res, ok = run(start)
    if not ok and X0 is not None:
        fell_back = True
        X, res, ok = run(block_jacobi_start(S, pat_x))
    if not ok:
        raise RuntimeError(f"Hotelling iteration did not converge: {res[-3:]}")
    return InverseResult(X, len(res), res, fell_back)


def inverse_error(X: BSM, S: BSM, pat_p: Pattern) -> Tuple[float, float, float]:
    """Truncation error of S^-1 (Sec. V.A): D = P_P(X S) - I; (mean |D|, max |D|, ||D||_F)."""
    XS, _ = spgemm(X, S, pat_p)
    D = axpby(1.0, XS, -1.0, identity(pat_p, X.b))
    a = np.abs(D.val)
    return float(a.mean()), float(a.max()), frob(D)


def taylor_propagator(A: BSM, dt: float, p: int, pat_u: Pattern) -> BSM:
    """U = sum_{n=0}^{p} T_n (Eq. matrix_exp, Eq. EM), truncated to pat_u at every product."""
    T = identity(pat_u, A.b)
    U = T.copy()
    if p >= 1:
        assert A.pat is pat_u
        T = BSM(pat_u, A.b, (-1j * dt) * A.val)
        U = axpby(1.0, U, 1.0, T)
    for n in range(2, p + 1):
        T, _ = spgemm(A, T, pat_u, alpha=-1j * dt / n)
        U = axpby(1.0, U, 1.0, T)
    return U


def hermitize(K: BSM) -> BSM:
    """K <- (K + K^dagger) / 2."""
    return BSM(K.pat, K.b, 0.5 * (K.val + K.conj_transpose().val))


def herm_error(K: BSM) -> float:
    """||K - K^dagger||_F / ||K||_F."""
    return frob(axpby(1.0, K, -1.0, K.conj_transpose())) / frob(K)


def mulliken(K: BSM, S: BSM) -> np.ndarray:
    """q_i = Re sum_j tr(K_ij S_ji) over the pairs kept in both K and S."""
    n = S.pat.n
    q = np.zeros(n)
    rs = S.pat.rows()
    cs = S.pat.col.astype(np.int64)
    pk = K.pat.index(rs, cs)                 # K_ij
    ps_t = S.pat.index(cs, rs)               # S_ji
    keep = pk >= 0
    tr = np.einsum("tab,tba->t", K.val[pk[keep]], S.val[ps_t[keep]])
    np.add.at(q, rs[keep], tr.real)
    return q


def centroid(xyz: np.ndarray) -> np.ndarray:
    """r_c = (sum_i r_i) / n, each coordinate sum rounded once (math.fsum is
    exactly rounded), so r_c does not depend on the order of the atoms."""
    n = xyz.shape[0]
    return np.array([math.fsum(xyz[:, k]) for k in range(3)]) / n


def dipole(q: np.ndarray, xyz: np.ndarray) -> np.ndarray:
    """P = -sum_i (r_i - r_c) q_i (electron charge -1, r_c = centroid)."""
    rc = centroid(xyz)
    return -((xyz - rc) * q[:, None]).sum(axis=0)


def kick(K: BSM, xyz: np.ndarray, kappa: Sequence[float]) -> BSM:
    """K_ij <- exp(i kappa . (r_i - r_j)) K_ij (impulsive limit of the field of Sec. II.B)."""
    kap = np.asarray(kappa, dtype=np.float64)
    r = K.pat.rows()
    c = K.pat.col.astype(np.int64)
    ph = np.exp(1j * ((xyz[r] - xyz[c]) @ kap))
    return BSM(K.pat, K.b, K.val * ph[:, None, None])


def add_onsite(H0: BSM, shift: np.ndarray) -> BSM:
    """H = H0 + diag(shift_i) on atom i's diagonal block."""
    H = H0.copy()
    d = H0.pat.index(np.arange(H0.pat.n), np.arange(H0.pat.n))
    H.val[d] += shift[:, None, None] * np.eye(H0.b)
    return H


def unitarity(U: BSM, S: BSM, pat_p: Pattern) -> Tuple[float, float, float]:
    """||P_P(U^dagger P_P(S U)) - S|| as (relative Frobenius, mean |.|, max |.|)."""
    V, _ = spgemm(S, U, pat_p)
    Z, _ = spgemm(U, V, pat_p, op_a=1)
    Sp = from_coo_bsm(S, pat_p)
    D = axpby(1.0, Z, -1.0, Sp)
    a = np.abs(D.val)
    return frob(D) / frob(S), float(a.mean()), float(a.max())


def from_coo_bsm(M: BSM, pat: Pattern) -> BSM:
    """Copy M onto a wider pattern (zeros where M has no block)."""
    out = zeros(pat, M.b)
    r = M.pat.rows()
    pos = pat.index(r, M.pat.col)
    assert np.all(pos >= 0)
    out.val[pos] = M.val
    return out


# ----------------------------------------------------------------------------
# a whole propagation
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Setup:
    xyz: np.ndarray
    b: int
    pat_hs: Pattern
    pat_p: Pattern
    pat_k: Pattern
    S: BSM
    H0: BSM
    K0: BSM


def setup(sys_) -> Setup:
    """Patterns and matrices of a generated system on the oracle's storage."""
    p_hs = pattern(sys_.xyz, sys_.R_HS)
    p_k = pattern(sys_.xyz, sys_.R_K)
    p_p = p_k if sys_.R_P == sys_.R_K else (p_hs if sys_.R_P == sys_.R_HS else pattern(sys_.xyz, sys_.R_P))
    S = from_coo(sys_.S, p_hs, sys_.b)
    H0 = from_coo(sys_.H0, p_hs, sys_.b)
    K0 = from_coo(sys_.K0, p_k, sys_.b)
    return Setup(sys_.xyz, sys_.b, p_hs, p_p, p_k, S, H0, K0)


@dataclasses.dataclass
class Field:
    """External field of Gaussian time profile (Sec. II.B, linear response):
    E(t) = E0 exp(-(t - t0)^2 / (2 sigma^2)).  The external potential is
    -E(t) . r; the electrons (charge -1) have the potential energy +E(t) . r,
    so an impulsive field of integral -kappa is the kick exp(i kappa . r)."""
    E0: Tuple[float, float, float]
    t0: float
    sigma: float

    def at(self, t: float) -> np.ndarray:
        return np.asarray(self.E0, dtype=np.float64) * np.exp(-(t - self.t0) ** 2 / (2.0 * self.sigma ** 2))


def field_term(S: BSM, xyz: np.ndarray, E: np.ndarray) -> BSM:
    """Matrix of the electrons' energy E . (r - r_c) on the support functions, in
    the position model of the dipole reading: <i|r|j> = (r_i + r_j)/2 S_ij,
    r_c the atom centroid."""
    rc = centroid(xyz)
    r = S.pat.rows()
    c = S.pat.col.astype(np.int64)
    mid = 0.5 * ((xyz[r] - rc) + (xyz[c] - rc))          # (nnzb, 3)
    return BSM(S.pat, S.b, (mid @ np.asarray(E, dtype=np.float64))[:, None, None] * S.val)


def hamiltonian(st: "Setup", q_eff: Optional[np.ndarray], q_ref: np.ndarray, t: float, h_model: str,
                h_gain: float, field: Optional[Field]) -> BSM:
    """H at time t: H0, plus g diag(q_eff - q_ref) for the Mulliken model, plus
    the external field term."""
    H = st.H0
    if h_model == "mulliken":
        H = add_onsite(H, h_gain * (q_eff - q_ref))
    if field is not None:
        H = axpby(1.0, H, 1.0, field_term(st.S, st.xyz, field.at(t)))
    return H


M4_THETA = (0.5 - np.sqrt(3.0) / 6.0, 0.5 + np.sqrt(3.0) / 6.0)


def complex_taylor(M: BSM, p: int, pat_u: Pattern) -> BSM:
    """U = sum_{n=0}^{p} T_n, T_0 = I, T_1 = M, T_n = P_U(M T_{n-1}) / n: the
    truncated Taylor series of exp(M) for a general (complex) exponent."""
    T = identity(pat_u, M.b)
    U = T.copy()
    if p >= 1:
        T = M.copy()
        U = axpby(1.0, U, 1.0, T)
    for n in range(2, p + 1):
        T, _ = spgemm(M, T, pat_u, alpha=1.0 / n)
        U = axpby(1.0, U, 1.0, T)
    return U


def build_u(kind: str, A_at, dt: float, p: int, pat_u: Pattern) -> BSM:
    """One step's propagator from A(theta) = P(X H(t + theta dt)) (Sec. II.A):

    * em   (Eq. EM):   exp(-i dt A(1/2))
    * etrs (ETRS):     exp(-i dt/2 A(1)) exp(-i dt/2 A(0)), product truncated to P_U
    * m4   (Magnus):   exp(M), M = -i dt/2 (A1 + A2) - (sqrt(3) dt^2 / 12) [A2, A1],
                       A_k = A(theta_k), theta_{1,2} = 1/2 -/+ sqrt(3)/6 (Gauss-Legendre),
                       commutator from the two truncated products.
    """
    if kind == "em":
        return taylor_propagator(A_at(0.5), dt, p, pat_u)
    if kind == "etrs":
        U1 = taylor_propagator(A_at(0.0), 0.5 * dt, p, pat_u)
        U2 = taylor_propagator(A_at(1.0), 0.5 * dt, p, pat_u)
        U, _ = spgemm(U2, U1, pat_u)
        return U
    if kind == "m4":
        A1, A2 = A_at(M4_THETA[0]), A_at(M4_THETA[1])
        C21, _ = spgemm(A2, A1, pat_u)
        C12, _ = spgemm(A1, A2, pat_u)
        comm = axpby(1.0, C21, -1.0, C12)
        M = axpby(-0.5j * dt, axpby(1.0, A1, 1.0, A2), -np.sqrt(3.0) * dt * dt / 12.0, comm)
        return complex_taylor(M, p, pat_u)
    raise ValueError(f"unknown propagator {kind}")


@dataclasses.dataclass
class Trace:
    rows: np.ndarray          # (n_steps, 6): t, Px, Py, Pz, Tr(KS), herm_err
    K: BSM
    U: BSM
    X: BSM
    inverse: InverseResult


def propagate(st: Setup, n_steps: int, dt: float, kappa: Sequence[float], h_model: str = "fixed",
              h_gain: float = 0.5, p: int = 5, X: Optional[InverseResult] = None,
              inv_tol: float = 1e-10, propagator: str = "em", field: Optional[Field] = None,
              sc_steps: int = 0, sc_iters: int = 0, t_start: float = 0.0,
              q_ref: Optional[np.ndarray] = None) -> Trace:
    """Kick K0 and take n steps (Secs. II.A, II.B, IV, V.A).

    The charges entering H at t + theta dt are extrapolated from the last two
    steps, q = q(t) + theta (q(t) - q(t - dt)) (predictor).  For the first
    sc_steps steps the step is repeated sc_iters more times with the charges
    interpolated between q(t) and the q(t + dt) of the previous pass,
    q = q(t) + theta (q(t + dt) - q(t)) (corrector; Sec. IV.A, self-consistent
    H_+).  The field's own time dependence is evaluated exactly, at
    t = t_start + (s + theta) dt in step s.  q_ref defaults to q(K0)."""
    inv = X if X is not None else hotelling(st.S, st.pat_p, tol=inv_tol)
    Xm = inv.X
    if q_ref is None:
        q_ref = mulliken(st.K0, st.S)
    K = kick(st.K0, st.xyz, kappa)
    q_cur = mulliken(K, st.S)
    q_prev = q_cur.copy()
    U = None
    rows = []
    varying = h_model == "mulliken" or field is not None
    for s in range(n_steps):
        t = t_start + s * dt
        passes = 1 + (sc_iters if s < sc_steps else 0)
        q_new = None
        for it in range(passes):
            if varying or U is None:
                if it == 0:
                    q_at = lambda th: q_cur + th * (q_cur - q_prev)
                else:
                    q_at = lambda th, qn=q_new: q_cur + th * (qn - q_cur)

                def A_at(th):
                    H = hamiltonian(st, q_at(th), q_ref, t + th * dt, h_model, h_gain, field)
                    return spgemm(Xm, H, st.pat_p)[0]

                U = build_u(propagator, A_at, dt, p, st.pat_p)
            W, _ = spgemm(U, K, st.pat_k)
            Kn, _ = spgemm(W, U, st.pat_k, op_b=1)
            he = herm_error(Kn)
            Kh = hermitize(Kn)
            q_new = mulliken(Kh, st.S)
        K = Kh
        q_prev, q_cur = q_cur, q_new
        P = dipole(q_cur, st.xyz)
        rows.append([t_start + (s + 1) * dt, P[0], P[1], P[2], q_cur.sum(), he])
    return Trace(np.asarray(rows).reshape(-1, 6), K, U, Xm, inv)


def spectrum(P: np.ndarray, P0: np.ndarray, dt: float, E: Optional[np.ndarray], kappa: Optional[np.ndarray],
             gamma: float, omegas: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Damped transform of the induced dipole (Sec. II.B, linear response).

    P: (n, 3) dipole after steps 1..n (times t_k = k dt); P0: dipole at t = 0.
    F[f](w) = sum_{k=0}^{n} f(t_k) exp((i w - gamma) t_k) dt.  The polarisability
    alpha_jj(w) = F[P_j - P0_j](w) / F[E_j](w) for a field along axis j; for a kick exp(i kappa . r) the
    field transform is -kappa_j (impulsive field of integral -kappa).  Returns
    alpha (n_w, 3) complex (NaN where direction j has no field) and the
    strength function S(w) = (2 w / pi) Im(sum_j alpha_jj / 3).
    """
    n = P.shape[0]
    t = dt * np.arange(n + 1)
    dP = np.vstack([np.zeros((1, 3)), P - P0[None, :]])
    ph = np.exp((1j * omegas[:, None] - gamma) * t[None, :]) * dt      # (n_w, n+1)
    FP = ph @ dP                                                        # (n_w, 3)
    if E is not None:
        FE = ph @ E                                                     # E: (n+1, 3) at t_k
    else:
        FE = np.broadcast_to(-np.asarray(kappa, dtype=np.float64), FP.shape).astype(complex)
    with np.errstate(divide="ignore", invalid="ignore"):
        alpha = np.where(np.abs(FE) > 0, FP / np.where(FE == 0, 1, FE), np.nan)
    tr = np.nansum(alpha, axis=1)
    return alpha, 2.0 * omegas / np.pi * np.imag(tr / 3.0)


# ----------------------------------------------------------------------------
# ground state by truncated trace-correcting purification
# ----------------------------------------------------------------------------

def trace(M: BSM) -> float:
    """Sum of the diagonal elements of the diagonal blocks (real part)."""
    d = M.pat.index(np.arange(M.pat.n), np.arange(M.pat.n))
    return float(np.real(np.einsum("kaa->", M.val[d])))


def gershgorin(A: BSM) -> Tuple[float, float]:
    """Bounds [lo, hi] on the eigenvalues of A from its Gershgorin row discs:
    a_ii -/+ sum_{j != i} |a_ij| over the stored blocks."""
    n, b = A.pat.n, A.b
    rowsum = np.zeros((n, b))
    np.add.at(rowsum, A.pat.rows(), np.abs(A.val).sum(axis=2))
    d = A.pat.index(np.arange(n), np.arange(n))
    cen = np.real(np.einsum("kaa->ka", A.val[d]))
    rad = rowsum - np.abs(cen)
    return float((cen - rad).min()), float((cen + rad).max())


@dataclasses.dataclass
class GroundState:
    K: BSM
    iters: int
    branches: int          # bit k set: iteration k took Z <- 2 Z - Z^2 (else Z <- Z^2)
    idempotency: List[float]


def ground_state(S: BSM, H: BSM, X: BSM, pat_p: Pattern, pat_k: Pattern, n_occ: float,
                 tol: float = 1e-10, max_iter: int = 100) -> GroundState:
    """Density matrix of the n_occ lowest states of H v = e S v, linear scaling
    (the ground state that precedes the propagation; Sec. II.A, K S K = K,
    Tr(K S) = n_occ), by trace-correcting purification (Niklasson 2002) of
    A = P_P(S^-1 H) with X ~ S^-1:

      Z_0 = (hi I - A) / (hi - lo), [lo, hi] the Gershgorin bounds of A;
      each iteration Z^2 = P_P(Z Z); stop when |Tr Z - Tr Z^2| <= tol n_occ, or
      when that measure stops falling below 1e-4 n_occ (the truncation floor),
      else Z <- Z^2 if Tr Z > n_occ, otherwise Z <- 2 Z - Z^2;
      K = P_K(Z X), symmetrised (K + K^T) / 2.

    Z tends to the projector K S on the occupied states, so Z S^-1 = K."""
    A, _ = spgemm(X, H, pat_p)
    lo, hi = gershgorin(A)
    Z = axpby(hi / (hi - lo), identity(pat_p, A.b), -1.0 / (hi - lo), A)
    hist: List[float] = []
    branches = 0
    it = 0
    for it in range(max_iter):
        Z2, _ = spgemm(Z, Z, pat_p)
        tz, tz2 = trace(Z), trace(Z2)
        idem = abs(tz - tz2)
        hist.append(idem)
        if idem <= tol * n_occ:
            break
        if it >= 1 and hist[-2] < 1e-4 * n_occ and idem >= hist[-2]:
            break
        if tz > n_occ:
            Z = Z2
        else:
            Z = axpby(2.0, Z, -1.0, Z2)
            branches |= 1 << it
    K, _ = spgemm(Z, X, pat_k)
    K = BSM(K.pat, K.b, 0.5 * (K.val + K.conj_transpose().val))
    return GroundState(K, len(hist), branches, hist)

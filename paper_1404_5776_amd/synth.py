"""Seeded synthetic workloads for truncated block-sparse density-matrix propagation.

This module only *draws inputs*: atom positions, the overlap S, the ground-state
Hamiltonian H0 and the starting density matrix K0, each as atom-pair blocks in
coordinate (COO) form.  It contains none of the propagation arithmetic (no
truncated products, no inverse, no propagator, no observables); the oracle and
the GPU library each build their own neighbour lists and do their own maths
from these arrays.

The paper's systems (molecules and alkane chains described with pseudo-atomic
orbital bases and a DFT Hamiltonian, Secs. III and V) cannot be reproduced
here, so these stand-ins keep their structure instead: atom-centred blocks of
b functions, matrices that vanish beyond a spatial cut-off (Sec. II.A), a
non-orthogonal overlap, a gapped Hamiltonian and the paper's time step of
0.05 a.u. (Sec. V.B).

Recipe (all lengths in bohr, energies in hartree):

* clusters: cube of side (N/0.026)^(1/3); random sequential addition of
  uniform points, keeping those at least 2.5 from every earlier point;
* lattices: diamond conventional cell with nearest-neighbour distance 3.37
  (a = 4*3.37/sqrt(3)), 8 atoms per cell, open boundaries, each Cartesian
  component displaced by N(0, (0.02*3.37)^2);
* atoms are emitted in Morton (Z-curve) order of a 3.37-bohr grid;
* S: S_ii = I_b; for a pair closer than R_HS, S_ij = exp(-(d/3.37)^2) U(-1,1)^{b x b},
  S_ji = S_ij^T; every off-diagonal block is then scaled by one factor so that
  the largest off-diagonal absolute row sum is 0.8 (so S is SPD with spectrum
  in [0.2, 1.8] by Gershgorin's theorem);
* H0: H_ii = diag(-gap/2 for the lowest floor(b/2) functions, +gap/2 otherwise)
  + eta*sym(U(-1,1)); H_ij = -t0 exp(-(d/3.37)^2) U(-1,1), symmetric;
  gap = 1.0, t0 = 0.05, eta = 0.05;
* K0 (real symmetric, kept only for pairs closer than R_K):
  - "exact": lowest floor(b/2)*N (N/2 for b = 1) eigenvectors V of the generalized problem
    H0 v = e S v (V^T S V = I), K0 = V V^T (spinless, so K0 S K0 = K0);
  - "local": for systems too large for a dense eigensolver, a
    divide-and-conquer density matrix (W. Yang, Phys. Rev. Lett. 66, 1438
    (1991)) with the simplest partition: atom i's row blocks come from the
    exact K0 of the sub-system of atoms within r_loc of i, and the result is
    symmetrized.  It is an approximate ground state, used as a realistic
    Hermitian starting point with the right sparsity and magnitude.

Every random draw comes from numpy.random.SeedSequence(seed) children, so a
(config, seed) pair fixes every byte.  Generation refuses geometries in which
any pair distance is within 1e-9 R^2 of a cut-off (in squared distance), so
that no two implementations can disagree on membership because of rounding.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
from scipy.spatial import cKDTree

NN_DIST = 3.37          # nearest-neighbour distance of the lattice (bohr)
DECAY_LEN = 3.37        # Gaussian decay length of off-diagonal blocks (bohr)
S_ROWSUM = 0.8          # largest off-diagonal absolute row sum of S
GAP = 1.0               # on-site splitting of H0 (hartree)
T0 = 0.05               # hopping scale of H0
ETA = 0.05              # on-site noise of H0
CLUSTER_DENSITY = 0.026  # atoms / bohr^3
CLUSTER_MIN_SEP = 2.5    # bohr
TIE_REL = 1e-9


@dataclasses.dataclass
class BlockCOO:
    """Atom-pair blocks of one matrix: data[t] is the (rows[t], cols[t]) block."""

    rows: np.ndarray   # (nnzb,) int32
    cols: np.ndarray   # (nnzb,) int32
    data: np.ndarray   # (nnzb, b, b) float64 or complex128

    @property
    def nnzb(self) -> int:
        return int(self.rows.shape[0])


@dataclasses.dataclass
class System:
    """One seeded synthetic system: geometry, cut-offs, S, H0, K0 and run settings."""

    name: str
    xyz: np.ndarray          # (N, 3) float64, bohr
    b: int                   # functions per atom (uniform)
    R_HS: float              # cut-off of H and S
    R_K: float               # cut-off of K
    R_P: float               # cut-off of S^-1, S^-1 H and U
    S: BlockCOO
    H0: BlockCOO
    K0: BlockCOO
    dt: float = 0.05
    n_steps: int = 100
    h_model: str = "fixed"   # "fixed" or "mulliken"
    h_gain: float = 0.5
    kappa: Tuple[float, float, float] = (0.01, 0.0, 0.0)
    k0_kind: str = "exact"
    seed: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nbf(self) -> np.ndarray:
        return np.full(self.n_atoms, self.b, dtype=np.int32)

    @property
    def n_basis(self) -> int:
        return self.n_atoms * self.b


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def _morton_key(cell: np.ndarray) -> np.ndarray:
    """Interleave the bits of non-negative integer grid coordinates (N,3)."""
    key = np.zeros(cell.shape[0], dtype=np.int64)
    c = cell.astype(np.int64)
    for bit in range(20):
        for ax in range(3):
            key |= ((c[:, ax] >> bit) & 1) << (3 * bit + ax)
    return key


def morton_order(xyz: np.ndarray, grid: float = NN_DIST) -> np.ndarray:
    lo = xyz.min(axis=0)
    cell = np.floor((xyz - lo) / grid).astype(np.int64)
    key = _morton_key(cell)
    return np.lexsort((np.arange(xyz.shape[0]), key))


def cluster_positions(n_atoms: int, rng: np.random.Generator,
                      density: float = CLUSTER_DENSITY,
                      min_sep: float = CLUSTER_MIN_SEP) -> np.ndarray:
    """Random sequential addition in a cube of side (N/density)^(1/3)."""
    side = (n_atoms / density) ** (1.0 / 3.0)
    pts: List[np.ndarray] = []
    grid = min_sep
    ncell = max(1, int(math.ceil(side / grid)))
    buckets: Dict[Tuple[int, int, int], List[int]] = {}
    tries = 0
    while len(pts) < n_atoms:
        tries += 1
        if tries > 2000 * n_atoms:
            raise RuntimeError("random sequential addition did not converge")
        p = rng.uniform(0.0, side, size=3)
        c = tuple(np.minimum((p // grid).astype(int), ncell - 1))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for q in buckets.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                        d = pts[q] - p
                        if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < min_sep * min_sep:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            buckets.setdefault(c, []).append(len(pts))
            pts.append(p)
    return np.asarray(pts, dtype=np.float64)


def diamond_positions(cells: Sequence[int], rng: np.random.Generator,
                      nn: float = NN_DIST, disp_frac: float = 0.02) -> np.ndarray:
    """Diamond lattice, 8 atoms per conventional cell, with Gaussian displacements."""
    a = 4.0 * nn / math.sqrt(3.0)
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                      [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])
    nx, ny, nz = cells
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    g = g.reshape(-1, 1, 3) + basis.reshape(1, 8, 3)
    xyz = (g.reshape(-1, 3) * a).astype(np.float64)
    xyz = xyz + rng.normal(0.0, disp_frac * nn, size=xyz.shape)
    return xyz


# ----------------------------------------------------------------------------
# pairs
# ----------------------------------------------------------------------------

def pairs_within(xyz: np.ndarray, R: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """All i<j with dx*dx+dy*dy+dz*dz < R*R (evaluated in float64 in that order)."""
    tree = cKDTree(xyz)
    pr = tree.query_pairs(r=R * (1.0 + 1e-6) + 1e-9, output_type="ndarray")
    if pr.size == 0:
        z = np.zeros(0, dtype=np.int64)
        return z, z, np.zeros(0)
    i = pr[:, 0].astype(np.int64)
    j = pr[:, 1].astype(np.int64)
    lo = np.minimum(i, j)
    hi = np.maximum(i, j)
    d = xyz[lo] - xyz[hi]
    d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    keep = d2 < R * R
    o = np.lexsort((hi[keep], lo[keep]))
    return lo[keep][o], hi[keep][o], d2[keep][o]


def check_no_ties(xyz: np.ndarray, radii: Sequence[float]) -> None:
    """Refuse a geometry with a squared pair distance within 1e-9 R^2 of R^2."""
    tree = cKDTree(xyz)
    for R in radii:
        pr = tree.query_pairs(r=R * 1.001 + 1e-6, output_type="ndarray")
        if pr.size == 0:
            continue
        d = xyz[pr[:, 0]] - xyz[pr[:, 1]]
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        if np.any(np.abs(d2 - R * R) < TIE_REL * R * R):
            raise ValueError(f"pair distance ties the cut-off R={R}")


# ----------------------------------------------------------------------------
# matrices
# ----------------------------------------------------------------------------

def _full_coo(n: int, lo: np.ndarray, hi: np.ndarray, diag: np.ndarray,
              off: np.ndarray) -> BlockCOO:
    """Symmetric block matrix from diagonal blocks and i<j blocks (j>i gets M^T)."""
    rows = np.concatenate([np.arange(n), lo, hi]).astype(np.int32)
    cols = np.concatenate([np.arange(n), hi, lo]).astype(np.int32)
    data = np.concatenate([diag, off, np.transpose(off, (0, 2, 1))], axis=0)
    o = np.lexsort((cols, rows))
    return BlockCOO(rows[o], cols[o], np.ascontiguousarray(data[o]))


def make_overlap(xyz, b, R_HS, rng) -> BlockCOO:
    n = xyz.shape[0]
    lo, hi, d2 = pairs_within(xyz, R_HS)
    d = np.sqrt(d2)
    off = np.exp(-(d / DECAY_LEN) ** 2)[:, None, None] * rng.uniform(-1.0, 1.0, size=(lo.size, b, b))
    rowsum = np.zeros((n, b))
    np.add.at(rowsum, lo, np.abs(off).sum(axis=2))
    np.add.at(rowsum, hi, np.abs(off).sum(axis=1))
    mx = rowsum.max() if rowsum.size else 0.0
    if mx > 0:
        off *= S_ROWSUM / mx
    diag = np.broadcast_to(np.eye(b), (n, b, b)).copy()
    return _full_coo(n, lo, hi, diag, off)


def make_hamiltonian(xyz, b, R_HS, rng) -> BlockCOO:
    n = xyz.shape[0]
    lo, hi, d2 = pairs_within(xyz, R_HS)
    d = np.sqrt(d2)
    onsite = np.where(np.arange(b) < b // 2, -0.5 * GAP, 0.5 * GAP)
    noise = rng.uniform(-1.0, 1.0, size=(n, b, b))
    diag = np.zeros((n, b, b))
    diag[:, np.arange(b), np.arange(b)] = onsite
    diag += ETA * 0.5 * (noise + np.transpose(noise, (0, 2, 1)))
    off = -T0 * np.exp(-(d / DECAY_LEN) ** 2)[:, None, None] * rng.uniform(-1.0, 1.0, size=(lo.size, b, b))
    return _full_coo(n, lo, hi, diag, off)


def coo_to_dense(m: BlockCOO, n_atoms: int, b: int) -> np.ndarray:
    """Dense (N*b, N*b) matrix from blocks (input helper for small systems)."""
    out = np.zeros((n_atoms * b, n_atoms * b), dtype=m.data.dtype)
    for t in range(m.nnzb):
        i, j = int(m.rows[t]), int(m.cols[t])
        out[i * b:(i + 1) * b, j * b:(j + 1) * b] = m.data[t]
    return out


def dense_to_coo(dense: np.ndarray, xyz: np.ndarray, b: int, R: float) -> BlockCOO:
    """Blocks of a dense matrix for the pairs closer than R, plus the diagonal."""
    n = xyz.shape[0]
    lo, hi, _ = pairs_within(xyz, R)
    rows = np.concatenate([np.arange(n), lo, hi]).astype(np.int32)
    cols = np.concatenate([np.arange(n), hi, lo]).astype(np.int32)
    o = np.lexsort((cols, rows))
    rows, cols = rows[o], cols[o]
    d4 = dense.reshape(n, b, n, b)
    data = np.ascontiguousarray(d4[rows, :, cols, :])
    return BlockCOO(rows, cols, data)


def n_occupied(n_atoms: int, b: int) -> int:
    """floor(b/2) occupied states per atom (half of all states for b = 1)."""
    return n_atoms * (b // 2) if b >= 2 else max(1, n_atoms // 2)


def k0_exact(S: BlockCOO, H0: BlockCOO, xyz, b, R_K) -> BlockCOO:
    from scipy.linalg import eigh
    n = xyz.shape[0]
    Sd = coo_to_dense(S, n, b)
    Hd = coo_to_dense(H0, n, b)
    nocc = n_occupied(n, b)
    w, V = eigh(Hd, Sd, subset_by_index=[0, nocc - 1])
    K = V @ V.T
    return dense_to_coo(0.5 * (K + K.T), xyz, b, R_K)


def k0_local(S: BlockCOO, H0: BlockCOO, xyz, b, R_K, r_loc: float = 4.5) -> BlockCOO:
    """Divide-and-conquer ground-state density matrix (see the module docstring)."""
    n = xyz.shape[0]
    assert r_loc < R_K
    tree = cKDTree(xyz)
    nbrs = tree.query_ball_point(xyz, r=r_loc)
    # block lookup for S and H0
    key_s = S.rows.astype(np.int64) * n + S.cols
    key_h = H0.rows.astype(np.int64) * n + H0.cols
    order_s = np.argsort(key_s)
    order_h = np.argsort(key_h)
    sk = key_s[order_s]
    hk = key_h[order_h]
    local = []
    for i in range(n):
        c = np.asarray(sorted(set(nbrs[i]) | {i}), dtype=np.int64)
        d = xyz[c] - xyz[i]
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        c = c[(d2 < r_loc * r_loc) | (c == i)]
        local.append(c)
    by_size: Dict[int, List[int]] = {}
    for i, c in enumerate(local):
        by_size.setdefault(len(c), []).append(i)
    acc: Dict[Tuple[int, int], np.ndarray] = {}
    for m, atoms in by_size.items():
        atoms = np.asarray(atoms)
        C = np.stack([local[i] for i in atoms])                # (g, m)
        ii = np.repeat(C, m, axis=1).reshape(-1)
        jj = np.tile(C, (1, m)).reshape(-1)
        keys = ii * n + jj
        ps = np.searchsorted(sk, keys)
        ph = np.searchsorted(hk, keys)
        ps = np.minimum(ps, sk.size - 1)
        ph = np.minimum(ph, hk.size - 1)
        has_s = sk[ps] == keys
        has_h = hk[ph] == keys
        Sb = np.where(has_s[:, None, None], S.data[order_s[ps]], 0.0)
        Hb = np.where(has_h[:, None, None], H0.data[order_h[ph]], 0.0)
        g = atoms.size
        Sl = Sb.reshape(g, m, m, b, b).transpose(0, 1, 3, 2, 4).reshape(g, m * b, m * b)
        Hl = Hb.reshape(g, m, m, b, b).transpose(0, 1, 3, 2, 4).reshape(g, m * b, m * b)
        # generalized symmetric eigenproblem through a Cholesky factor of S
        L = np.linalg.cholesky(Sl)
        Li = np.linalg.inv(L)
        Ht = Li @ Hl @ np.transpose(Li, (0, 2, 1))
        Ht = 0.5 * (Ht + np.transpose(Ht, (0, 2, 1)))
        w, Y = np.linalg.eigh(Ht)
        nocc = n_occupied(m, b)
        V = np.transpose(Li, (0, 2, 1)) @ Y[:, :, :nocc]
        Kl = V @ np.transpose(V, (0, 2, 1))                    # (g, mb, mb)
        for gi, i in enumerate(atoms):
            ci = local[i]
            pos = int(np.nonzero(ci == i)[0][0])
            rowblk = Kl[gi, pos * b:(pos + 1) * b, :]
            for q, j in enumerate(ci):
                blk = rowblk[:, q * b:(q + 1) * b]
                acc[(i, int(j))] = acc.get((i, int(j)), 0.0) + 0.5 * blk
                acc[(int(j), i)] = acc.get((int(j), i), 0.0) + 0.5 * blk.T
    keys = sorted(acc.keys())
    rows = np.array([k[0] for k in keys], dtype=np.int32)
    cols = np.array([k[1] for k in keys], dtype=np.int32)
    data = np.stack([acc[k] for k in keys]).astype(np.float64)
    return BlockCOO(rows, cols, data)


# ----------------------------------------------------------------------------
# systems
# ----------------------------------------------------------------------------

def _children(seed: int, n: int) -> List[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def build_system(name: str, xyz: np.ndarray, b: int, R_HS: float, R_K: float,
                 seed: int, k0: str = "auto", R_P: Optional[float] = None,
                 **run) -> System:
    """Assemble S, H0 and K0 for given positions (positions reordered to Morton order)."""
    xyz = np.ascontiguousarray(xyz[morton_order(xyz)])
    if R_P is None:
        R_P = max(R_K, R_HS)
    check_no_ties(xyz, sorted({R_HS, R_K, R_P}))
    r_s, r_h, _ = _children(seed + 7919, 3)
    S = make_overlap(xyz, b, R_HS, r_s)
    H0 = make_hamiltonian(xyz, b, R_HS, r_h)
    if k0 == "auto":
        k0 = "exact" if xyz.shape[0] * b <= 3000 else "local"
    if k0 == "exact":
        K0 = k0_exact(S, H0, xyz, b, R_K)
    elif k0 == "local":
        K0 = k0_local(S, H0, xyz, b, R_K)
    else:
        raise ValueError(k0)
    return System(name=name, xyz=xyz, b=b, R_HS=R_HS, R_K=R_K, R_P=R_P,
                  S=S, H0=H0, K0=K0, k0_kind=k0, seed=seed, **run)


def random_cluster(n_atoms: int, b: int, R_HS: float, R_K: float, seed: int,
                   **kw) -> System:
    (r_pos,) = _children(seed, 1)
    xyz = cluster_positions(n_atoms, r_pos)
    return build_system(f"cluster{n_atoms}_b{b}", xyz, b, R_HS, R_K, seed, **kw)


def diamond_lattice(cells: Sequence[int], b: int, R_HS: float, R_K: float,
                    seed: int, **kw) -> System:
    (r_pos,) = _children(seed, 1)
    xyz = diamond_positions(cells, r_pos)
    n = xyz.shape[0]
    return build_system(f"diamond{n}_b{b}", xyz, b, R_HS, R_K, seed, **kw)


# The five workloads.  Their exact readings are documented in the design notes.

def config1(seed: int = 1) -> System:
    """64-atom cluster, b=4, R_HS 8, R_K 12, exact K0, fixed H, 100 steps."""
    return random_cluster(64, 4, 8.0, 12.0, seed, k0="exact",
                          n_steps=100, h_model="fixed")


def config2(seed: int = 2, cells=(8, 8, 8), n_steps: int = 500, k0: str = "auto") -> System:
    """4,096-atom diamond lattice, b=13, R_HS 10, R_K 16, Mulliken H, 500 steps."""
    return diamond_lattice(cells, 13, 10.0, 16.0, seed, k0=k0,
                           n_steps=n_steps, h_model="mulliken")


def config3(R_K: float, seed: int = 3, cells=(16, 16, 16), n_steps: int = 1000) -> System:
    """32,768-atom lattice, b=4, R_HS 10, R_K in {8, 12, 16, 20}, Mulliken H."""
    return diamond_lattice(cells, 4, 10.0, R_K, seed, n_steps=n_steps, h_model="mulliken")


def config4_sizes(seed: int = 4, n_clusters: int = 64) -> List[Tuple[int, int]]:
    """(atoms, b) per cluster: log-uniform 50..2000 atoms, b in {4, 13} 50/50."""
    (rng,) = _children(seed, 1)
    n = np.exp(rng.uniform(math.log(50), math.log(2000), size=n_clusters)).astype(int)
    bs = np.where(rng.uniform(size=n_clusters) < 0.5, 4, 13)
    return [(int(a), int(b)) for a, b in zip(n, bs)]


def config4_cluster(k: int, seed: int = 4) -> System:
    sizes = config4_sizes(seed)
    n, b = sizes[k]
    return random_cluster(n, b, 8.0, 12.0, seed * 1000 + k, n_steps=100, h_model="fixed")


def _one_blas_thread():
    """Worker set-up: one BLAS thread per process (the pool supplies the parallelism)."""
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def config4_all(seed: int = 4, n_clusters: int = 64, workers: int = 0) -> List[System]:
    """The first n_clusters clusters of the 64-cluster list, generated in
    worker processes (spawned, so a parent that already uses the GPU is not
    forked); workers 0 means one per CPU, at most 16."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    if workers == 1 or n_clusters <= 1:
        return [config4_cluster(k, seed) for k in range(n_clusters)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                initializer=_one_blas_thread) as ex:
        # largest first, so the long ones do not finish last
        sizes = config4_sizes(seed)[:n_clusters]
        order = sorted(range(n_clusters), key=lambda k: -sizes[k][0] * sizes[k][1])
        futs = {k: ex.submit(config4_cluster, k, seed) for k in order}
        return [futs[k].result() for k in range(n_clusters)]


def config5(seed: int = 5, cells=(16, 16, 32), n_steps: int = 100) -> System:
    """65,536-atom lattice, b=4, R_HS 10, R_K 12, Mulliken H."""
    return diamond_lattice(cells, 4, 10.0, 12.0, seed, n_steps=n_steps, h_model="mulliken")


# ----------------------------------------------------------------------------
# per-atom block sizes (e.g. 4 functions on some elements, 13 on others)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class MixedCOO:
    """Atom-pair blocks of per-atom sizes: block t is nbf[rows[t]] x
    nbf[cols[t]], row-major; the blocks are concatenated in data."""

    rows: np.ndarray   # (nnzb,) int32
    cols: np.ndarray   # (nnzb,) int32
    data: np.ndarray   # (sum of block sizes,) float64

    @property
    def nnzb(self) -> int:
        return int(self.rows.shape[0])


@dataclasses.dataclass
class MixedSystem:
    """A system whose atoms carry different numbers of functions."""

    name: str
    xyz: np.ndarray
    nbf: np.ndarray          # (N,) int32
    R_HS: float
    R_K: float
    R_P: float
    S: MixedCOO
    H0: MixedCOO
    K0: MixedCOO
    dt: float = 0.05
    n_steps: int = 20
    h_model: str = "fixed"
    h_gain: float = 0.5
    kappa: Tuple[float, float, float] = (0.01, 0.0, 0.0)
    seed: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.nbf)]).astype(np.int64)


def dense_to_mixed(dense: np.ndarray, xyz: np.ndarray, nbf: np.ndarray, R: float) -> MixedCOO:
    """Blocks of a dense matrix (functions ordered atom by atom) for the pairs
    closer than R, plus the diagonal, in row-major pair order."""
    n = xyz.shape[0]
    off = np.concatenate([[0], np.cumsum(nbf)])
    lo, hi, _ = pairs_within(xyz, R)
    rows = np.concatenate([np.arange(n), lo, hi]).astype(np.int32)
    cols = np.concatenate([np.arange(n), hi, lo]).astype(np.int32)
    o = np.lexsort((cols, rows))
    rows, cols = rows[o], cols[o]
    data = np.concatenate([dense[off[i]:off[i + 1], off[j]:off[j + 1]].ravel() for i, j in zip(rows, cols)])
    return MixedCOO(rows, cols, data)


def mixed_cluster(n_atoms: int, seed: int, R_HS: float = 8.0, R_K: float = 12.0, sizes=(4, 13),
                  h_model: str = "fixed", n_steps: int = 20) -> MixedSystem:
    """Random cluster (config-1 density and spacing) whose atoms carry
    sizes[0] or sizes[1] functions (equal odds); S, H0 with the same
    Gaussian-decaying random blocks as the equal-size systems, K0 the
    occupied projector of the generalised eigenproblem (sum of floor(nbf/2)
    states), cut to R_K."""
    from scipy.linalg import eigh
    r_pos, r_b, r_s, r_h = _children(seed, 4)
    xyz = cluster_positions(n_atoms, r_pos)
    xyz = np.ascontiguousarray(xyz[morton_order(xyz)])
    check_no_ties(xyz, sorted({R_HS, R_K}))
    nbf = np.where(r_b.uniform(size=n_atoms) < 0.5, sizes[0], sizes[1]).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(nbf)])
    nf = int(off[-1])
    lo, hi, d2 = pairs_within(xyz, R_HS)
    decay = np.exp(-(np.sqrt(d2) / DECAY_LEN) ** 2)
    # overlap: unit diagonal blocks, off-diagonal blocks scaled to row sums S_ROWSUM at most
    S = np.eye(nf)
    for t, (i, j) in enumerate(zip(lo, hi)):
        S[off[i]:off[i + 1], off[j]:off[j + 1]] = decay[t] * r_s.uniform(-1.0, 1.0, size=(nbf[i], nbf[j]))
    up = np.triu(S, 1)
    S = np.eye(nf) + up + up.T
    rs = np.abs(S - np.eye(nf)).sum(axis=1).max()
    if rs > 0:
        S = np.eye(nf) + (S - np.eye(nf)) * (S_ROWSUM / rs)
    # Hamiltonian: split on-site levels plus symmetric noise, hopping -T0 decay U(-1, 1)
    H = np.zeros((nf, nf))
    for i in range(n_atoms):
        b = nbf[i]
        lev = np.where(np.arange(b) < b // 2, -0.5 * GAP, 0.5 * GAP)
        nz = r_h.uniform(-1.0, 1.0, size=(b, b))
        H[off[i]:off[i + 1], off[i]:off[i + 1]] = np.diag(lev) + ETA * 0.5 * (nz + nz.T)
    for t, (i, j) in enumerate(zip(lo, hi)):
        blk = -T0 * decay[t] * r_h.uniform(-1.0, 1.0, size=(nbf[i], nbf[j]))
        H[off[i]:off[i + 1], off[j]:off[j + 1]] = blk
        H[off[j]:off[j + 1], off[i]:off[i + 1]] = blk.T
    nocc = int(sum(b // 2 for b in nbf))
    _, V = eigh(H, S, subset_by_index=[0, nocc - 1])
    K = V @ V.T
    K = 0.5 * (K + K.T)
    return MixedSystem(name=f"mixed{n_atoms}", xyz=xyz, nbf=nbf, R_HS=R_HS, R_K=R_K, R_P=max(R_HS, R_K),
                       S=dense_to_mixed(S, xyz, nbf, R_HS), H0=dense_to_mixed(H, xyz, nbf, R_HS),
                       K0=dense_to_mixed(K, xyz, nbf, R_K), h_model=h_model, n_steps=n_steps, seed=seed)


# ----------------------------------------------------------------------------
# free-standing random operands for product-level tests
# ----------------------------------------------------------------------------

def random_blocks(rows: np.ndarray, cols: np.ndarray, b: int, seed: int,
                  complex_: bool) -> np.ndarray:
    """U(-1,1) blocks for a given list of pairs (real or complex128)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=(rows.size, b, b))
    if not complex_:
        return re
    im = rng.uniform(-1.0, 1.0, size=(rows.size, b, b))
    return re + 1j * im


def pattern_coo(xyz: np.ndarray, R: float) -> Tuple[np.ndarray, np.ndarray]:
    """(rows, cols) of all pairs closer than R plus the diagonal, row-major sorted."""
    n = xyz.shape[0]
    lo, hi, _ = pairs_within(xyz, R)
    rows = np.concatenate([np.arange(n), lo, hi]).astype(np.int32)
    cols = np.concatenate([np.arange(n), hi, lo]).astype(np.int32)
    o = np.lexsort((cols, rows))
    return rows[o], cols[o]

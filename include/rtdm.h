/*
 * rtdm.h -- truncated block-sparse density-matrix RT-TDDFT propagation on one
 * AMD Instinct MI355X (gfx950).
 *
 * The library evolves the auxiliary density matrix K of a linear-scaling DFT
 * code under the quantum Liouville equation in a non-orthogonal basis
 * (O'Rourke & Bowler, arXiv:1404.5776, Sec. II.A):
 *
 *     i dK/dt = S^-1 H K - K H S^-1,   K(t+dt) = U K(t) U^dagger,
 *     U = exp(-i S^-1 H(t+dt/2) dt)          (exponential midpoint, Eq. EM)
 *
 * with the exponential taken as a truncated Taylor series (Eq. matrix_exp,
 * Sec. IV.B), S^-1 from Hotelling's iteration (Sec. V.A), and every matrix and
 * every product truncated to a spatial cut-off radius on atom pairs
 * (Sec. II.A, Sec. V.A, Sec. V.B).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status: RTDM_OK (0) or a negative RTDM_E_*
 *   code.  No C++ exception crosses this boundary.  rtdm_last_error(ctx)
 *   returns a message for the last failing call on ctx (valid until the next
 *   call on ctx).
 * - A context is not thread-safe: use one context per host thread.
 * - Atomic units: positions in bohr, time in a.u. (hbar = 1), energies in Ha.
 * - Atoms keep the caller's order.  Matrices are stored in atom-pair blocks;
 *   block (i, j) of a matrix of range R exists iff i == j or
 *   dx*dx + dy*dy + dz*dz < R*R (double precision, no periodic images).
 * - Blocks passed across the boundary are b x b row-major.  Complex data is
 *   interleaved (re, im) double pairs ("complex128"); real data is double.
 * - Host buffers stay owned by the caller and are copied; device buffers
 *   passed in are read (or written) during the call on the given stream.
 *   Device memory for the library's own state is allocated by the library
 *   (hipMalloc) in set_ranges / upload / build_inverse and freed by
 *   rtdm_destroy; rtdm_step allocates only when its observable buffer must
 *   grow.
 * - `hip_stream` is a hipStream_t (NULL = the device's null stream).  Calls
 *   that take a stream enqueue work on it and return without waiting, except
 *   those documented as synchronising (they return host scalars).
 */
#ifndef RTDM_H
#define RTDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtdm_ctx rtdm_ctx;

/* Status codes. */
enum {
    RTDM_OK = 0,
    RTDM_E_ARG = -1,          /* bad argument (size, pointer, enum value) */
    RTDM_E_STATE = -2,        /* call out of order (e.g. step before build_inverse) */
    RTDM_E_OOM = -3,          /* device or host allocation failed */
    RTDM_E_HIP = -4,          /* a HIP runtime call failed */
    RTDM_E_NOCONV = -5,       /* Hotelling iteration did not converge */
    RTDM_E_NUMERIC = -6,      /* non-finite value detected */
    RTDM_E_UNSUPPORTED = -7   /* valid request the library does not implement */
};

/* Matrix slots.  Range and value type of each slot:
 *   S, H0, H : R_HS, real symmetric (S: overlap, Sec. II.A; H0: Hamiltonian
 *              as uploaded; H: the Hamiltonian used by the last propagator
 *              build, H0 plus the on-site model shift)
 *   X        : R_P,  real, the truncated inverse overlap (Sec. V.A)
 *   A        : R_P,  real, the truncated product S^-1 H (Sec. V.A)
 *   U        : R_P,  complex, the Taylor propagator (Eq. EM, Eq. matrix_exp)
 *   K        : R_K,  complex Hermitian, the density matrix (Sec. II.A)
 *   W        : R_K,  complex, the intermediate U K of the last step
 * For tests, any slot may be uploaded and used as an operand of rtdm_multiply. */
typedef enum {
    RTDM_MAT_S = 0,
    RTDM_MAT_H0 = 1,
    RTDM_MAT_H = 2,
    RTDM_MAT_X = 3,
    RTDM_MAT_A = 4,
    RTDM_MAT_U = 5,
    RTDM_MAT_K = 6,
    RTDM_MAT_W = 7,
    RTDM_MAT_COUNT = 8
} rtdm_mat;

/* The truncated products of one step and of the inverse iteration. */
typedef enum {
    RTDM_PROD_XH = 0,   /* A = P_P(X H)                  (Sec. V.A)            */
    RTDM_PROD_AT = 1,   /* T_n = P_P(c A T_{n-1})        (Eq. matrix_exp)      */
    RTDM_PROD_UK = 2,   /* W = P_K(U K)                  (Sec. II.A solution)  */
    RTDM_PROD_WU = 3,   /* K' = P_K(W U^dagger)          (Sec. II.A solution)  */
    RTDM_PROD_SX = 4,   /* P_P(S X), also P_P(S U)       (Sec. V.A, Sec. IV)   */
    RTDM_PROD_UV = 5,   /* P_P(U^dagger V)               (Sec. IV, Eq. s_unit) */
    RTDM_PROD_ZX = 6,   /* P_K(Z X), Z on R_P            (ground state, rtdm_ground_state) */
    RTDM_PROD_COUNT = 7
} rtdm_prod;

/* Arithmetic of the block products of rtdm_step and rtdm_multiply:
 *   FP64        FP64 matrix cores;
 *   FP32        every product on FP32 matrix cores with FP32 accumulation;
 *   FP32_TAYLOR only the Taylor-term products T_n = P(c A T_{n-1}) with
 *               n >= taylor_low_from in FP32 (their norms shrink like
 *               (dt |A|)^n / n!, so their rounding enters U scaled down); the
 *               terms are stored in FP32 and summed into U in FP64;
 *               A = P(X H), U K and W U^dagger stay FP64.
 *   BF16X3      every block product split-precision on the BF16 matrix
 *               cores: x = hi + lo with hi = bf16(x), lo = bf16(x - hi),
 *               a b ~ ah bh + ah bl + al bh accumulated in FP32 (three-term
 *               split of Henry, Tang and Heinecke, 2019);
 *   FP16X2      every block product split on the FP16 matrix cores with a
 *               power-of-two scale s per operand matrix (max |x s| in
 *               [2^13, 2^14)): hi = fp16(x s), lo = fp16((x s - hi) 2^11),
 *               a b ~ (ah bh + (ah bl + al bh) 2^-11) / (sa sb), FP32
 *               accumulation (scaled split of Ootomo and Yokota, 2022).
 *   BF16X3_TAYLOR, FP16X2_TAYLOR  only the Taylor-term products with
 *               n >= taylor_low_from in that split form (FP64 storage).
 * Reduced-precision forms need b = 4 or 13.  Storage, reductions,
 * observables, the inverse iteration and the unitarity check always run in
 * FP64. */
enum {
    RTDM_PREC_FP64 = 0,
    RTDM_PREC_FP32 = 1,
    RTDM_PREC_FP32_TAYLOR = 2,
    RTDM_PREC_BF16X3 = 3,
    RTDM_PREC_FP16X2 = 4,
    RTDM_PREC_BF16X3_TAYLOR = 5,
    RTDM_PREC_FP16X2_TAYLOR = 6
};
enum { RTDM_HMODEL_FIXED = 0, RTDM_HMODEL_MULLIKEN = 1 };
/* Starting guess of the inverse iteration: block-Jacobi blockdiag(S_ii^-1);
 * cold I / (largest absolute row sum of S); the current X; or the learned
 * guess (rtdm_mlp_*): for every block of S's range, 2 delta_ij I - S_ij plus
 * the network's correction, zero elsewhere.  PREVIOUS and LEARNED fall back
 * to block-Jacobi when the iteration diverges from them. */
enum { RTDM_INV_BLOCK_JACOBI = 0, RTDM_INV_COLD = 1, RTDM_INV_PREVIOUS = 2, RTDM_INV_LEARNED = 3 };
/* Propagator of one step (Sec. II.A), with A(theta) = P_P(X H(t + theta dt)):
 *   EM    exponential midpoint (Eq. EM): U = exp(-i dt A(1/2));
 *   ETRS  enforced time-reversal symmetry: U = P_P(exp(-i dt/2 A(1)) exp(-i dt/2 A(0)));
 *   M4    fourth-order Magnus with two Gauss-Legendre points
 *         theta_{1,2} = 1/2 -/+ sqrt(3)/6: U = exp(M),
 *         M = -i dt/2 (A_1 + A_2) - (sqrt(3) dt^2 / 12) (P_P(A_2 A_1) - P_P(A_1 A_2)).
 * Each exponential is the truncated Taylor series of order taylor_order with
 * every product truncated to R_P (EM and ETRS: real recursion on A; M4:
 * complex recursion T_n = P_P(M T_{n-1}) / n).  ETRS and M4 need
 * RTDM_PREC_FP64.  Charges entering H(t + theta dt): extrapolated
 * q(t) + theta (q(t) - q(t - dt)); in the first sc_steps steps after a kick
 * the step is repeated sc_iters times with q(t) + theta (q(t + dt) - q(t)),
 * q(t + dt) from the previous pass (self-consistent H, Sec. IV.A). */
enum { RTDM_PROP_EM = 0, RTDM_PROP_ETRS = 1, RTDM_PROP_M4 = 2 };

/* Options of a context (rtdm_default_options fills the defaults). */
typedef struct {
    int taylor_order;      /* p: Taylor orders 0..p of the exponential (Sec. IV.B: six terms -> 5) */
    int unit_check_every;  /* m > 0: record ||U^dagger S U - S|| every m steps; 0: never */
    int precision;         /* RTDM_PREC_* (block products only) */
    int h_model;           /* RTDM_HMODEL_FIXED: H = H0; MULLIKEN: H = H0 + g diag(q_mid - q_ref) */
    double h_gain;         /* g of the on-site model (default 0.5) */
    int inv_start;         /* starting guess of the inverse iteration (default block-Jacobi) */
    double inv_tol;        /* stop when ||X_{k+1}-X_k||_F / ||X_{k+1}||_F <= tol (default 1e-10) */
    int inv_max_iter;      /* iteration cap (default 50) */
    int taylor_low_from;   /* *_TAYLOR precisions: first Taylor order n in reduced precision (>= 2, default 3) */
    int use_graph;         /* 1: rtdm_step replays captured HIP graphs of its steps (default 0) */
    int propagator;        /* RTDM_PROP_* (default EM) */
    int sc_steps;          /* steps after a kick with corrector passes (default 0) */
    int sc_iters;          /* corrector passes per such step (default 2) */
    double unit_tol;       /* > 0: at each unitarity check, stop with RTDM_E_NUMERIC when the relative
                              unitarity error exceeds it or Tr(KS) is not finite (default 0: record only) */
    int graph_steps;       /* use_graph: steps captured per graph (1..1024, default 16); a call replays
                              one graph per whole group of graph_steps steps and the one-step graph for
                              the rest (always the one-step graph while unit_check_every > 0) */
    int n_kicks;           /* kick sets (1..8, default 1): K matrices propagated side by side with one
                              shared propagator per step (rtdm_apply_kicks, rtdm_select_kick); more than
                              one needs h_model FIXED and sc_steps 0, since U must not depend on K */
    int xh_every_step;     /* MULLIKEN: 1 forms A(theta) = P_P(X H(t + theta dt)) by the full block product at
                              every time point (the cost of a Hamiltonian that changes everywhere); 0
                              (default) forms it as A0 + X D with A0 = P_P(X H0), built once while X and H0
                              stay unchanged, and D the diagonal on-site term, which scales block columns of
                              X: equal in exact arithmetic, rounded differently (FP64 products without a
                              field; otherwise always the full product) */
} rtdm_options;

/* Fill *opt with the defaults above.  Never fails for a non-NULL opt. */
int rtdm_default_options(rtdm_options *opt);

/* Create a context on HIP device `hip_device` (opt NULL = defaults).
 * *out receives the context; the caller releases it with rtdm_destroy.
 * Kernel-shape variables read from the environment at creation (for
 * measurements; results differ only in the order of the contraction sums):
 *   RTDM_RUN_REAL   outputs per row run of the real b = 13 step products (1 to 4, or 8; default 2)
 *   RTDM_RUN_CPLX   the same for the complex ones (1 to 4; default 2)
 *   RTDM_RUN_B4     b = 4 products over row runs of 16 outputs (16, default) or per-output lists (1)
 *   RTDM_ROW_TILE   rows per output tile of the b = 13 processing order (default 256)
 * A run length outside these values fails with RTDM_E_ARG. */
int rtdm_create(rtdm_ctx **out, int hip_device, const rtdm_options *opt);

/* Release every host and device resource of ctx (NULL is accepted). */
int rtdm_destroy(rtdm_ctx *ctx);

/* Set the atoms: xyz[n][3] (bohr, host, copied) and nbf[n] functions per atom
 * (each in 1..16; the basis may differ per element, Sec. III).  With unequal
 * sizes the largest must be 4 or 13: every block is stored padded to that
 * size b, S and X carry the identity on an atom's padded functions and every
 * other matrix zeros, so the padded functions never mix with the atom's own
 * (all products act on them as on a separate identity block) and the
 * results on the real functions are those of the unpadded method.  The
 * on-site term of the Mulliken H leaves the padded functions out; the
 * field's term reaches them only through the padded identity of S, where it
 * stays on its own diagonal (K is zero there, so it changes nothing).  Mixed
 * sizes need FP64 products and the block-Jacobi or previous inverse start
 * (RTDM_E_UNSUPPORTED otherwise, and for the ground state and training
 * samples); every propagator, the corrector and the field run.  The
 * caller's blocks are then nbf_i x nbf_j (row-major) in every upload and
 * download.  Invalidates ranges, matrices and schedules. */
int rtdm_set_geometry(rtdm_ctx *ctx, int64_t n_atoms, const double *xyz, const int32_t *nbf);

/* Set the cut-off radii (Sec. II.A, Sec. V.A): R_HS for S and H, R_P for
 * S^-1, S^-1 H and U, R_K for K (R_P <= 0 selects max(R_HS, R_K)).  Builds the
 * neighbour lists of each range and the symbolic schedules (on the device;
 * the triple counts are then fixed) of the step's and the inverse's products
 * (XH, AT, UK, WU, SX), and of UV when the options check unitarity during
 * steps, so that rtdm_step allocates nothing.  UV otherwise (first
 * rtdm_unitarity or rtdm_observables after a step) and ZX (first
 * rtdm_ground_state) are scheduled on first use, in a bound workspace from
 * its reserve (RTDM_E_OOM when that is too small).  Zeroes every matrix.
 * Synchronises the device. */
int rtdm_set_ranges(rtdm_ctx *ctx, double R_HS, double R_P, double R_K);

/* Pattern of a slot's range: CSR over atoms, *row_ptr has n+1 entries and
 * *col_idx has *nnzb ascending atom indices per row.  Host pointers owned by
 * ctx, valid until the next set_geometry / set_ranges / destroy. */
int rtdm_pattern(rtdm_ctx *ctx, rtdm_mat mat, int64_t *n_rows, int64_t *nnzb,
                 const int64_t **row_ptr, const int32_t **col_idx);

/* Upload a slot from blocks in rtdm_pattern order (nnzb blocks of b*b, or of
 * nbf_i*nbf_j with mixed sizes, host data only).
 * is_complex: 1 = complex128 interleaved, 0 = double.  is_device: data is a
 * device pointer (1) or host pointer (0).  Real slots (S, H0, H, X, A) refuse
 * complex data whose imaginary part is not zero (RTDM_E_UNSUPPORTED).
 * Host uploads synchronise the stream before returning. */
int rtdm_upload(rtdm_ctx *ctx, rtdm_mat mat, const void *data, int is_complex,
                int is_device, void *hip_stream);

/* Upload a slot from host blocks in any order: rows[t], cols[t] name the
 * atom pair of block t (nnzb blocks of b*b, or nbf_i*nbf_j with mixed sizes,
 * concatenated; complex128 if is_complex else double).  Blocks absent from the list are zero; a pair outside the slot's
 * range is RTDM_E_ARG.  Synchronises the stream. */
int rtdm_upload_coo(rtdm_ctx *ctx, rtdm_mat mat, int64_t nnzb, const int32_t *rows,
                    const int32_t *cols, const void *data, int is_complex, void *hip_stream);

/* Download a slot as complex128 interleaved blocks in rtdm_pattern order
 * (real slots get zero imaginary parts) into dst (host or device; with mixed
 * sizes host only, blocks of nbf_i*nbf_j concatenated).
 * Synchronises the stream. */
int rtdm_download(rtdm_ctx *ctx, rtdm_mat mat, void *dst, int is_device, void *hip_stream);

/* The impulsive limit of the field of Sec. II.B on K:
 * K_ij <- exp(i kappa . (r_i - r_j)) K_ij.  Records q_ref = Mulliken charges
 * of K before the kick (if not recorded since the last K upload) and resets
 * the observable trace and the charge history of the midpoint extrapolation. */
int rtdm_apply_kick(rtdm_ctx *ctx, const double kappa[3], void *hip_stream);

/* Truncated Hotelling inverse of S (Sec. V.A):
 * X_{k+1} = P_P(2 X_k - X_k P_P(S X_k)) from the options' starting guess,
 * until ||X_{k+1}-X_k||_F/||X_{k+1}||_F <= inv_tol.  A residual that rises
 * after the first iteration or is not finite falls back to the block-Jacobi
 * start when the guess was RTDM_INV_PREVIOUS, else returns RTDM_E_NOCONV.
 * iters / residual (may be NULL) receive the iteration count and last
 * residual.  Synchronises (one scalar read per iteration). */
int rtdm_build_inverse(rtdm_ctx *ctx, void *hip_stream, int *iters, double *residual);

/* n_steps steps of length dt (Sec. II.A, Eq. EM, Eq. matrix_exp): per step
 * H at the propagator's time points (options' model and field), A = P_P(X H),
 * the Taylor propagator U on R_P (RTDM_PROP_*), W = P_K(U K),
 * K' = P_K(W U^dagger), K <- (K' + K'^dagger)/2, then the observables of the
 * new K appended to the trace.  With a fixed H and no field the propagator of
 * the first step is reused.  Asynchronous on hip_stream. */
int rtdm_step(rtdm_ctx *ctx, double dt, int64_t n_steps, void *hip_stream);

/* Batches of contexts (Sec. II.B: independent propagations, e.g. many systems
 * and their x/y/z kicks, advanced together).  A batch steps every member
 * context n_steps times per rtdm_batch_step call with the same dt: whole
 * groups of graph_steps steps replay one captured HIP graph in which every
 * context's steps run on a capture branch of their own (so the contexts'
 * kernels may overlap), launched on hip_stream (when NULL, on a stream of
 * the batch's that is ordered with the null stream); steps that a captured step cannot repeat (a fixed H's first
 * step, corrector passes after a kick) and the remainder of n_steps run
 * eagerly.  Every context then holds what n_steps calls of rtdm_step would
 * have left (tested bit for bit).  The graph is captured again when dt
 * changes or a member's own captured steps turn stale.
 *   create: ctxs = 1..64 distinct contexts of one device (the batch keeps the
 *           pointers; destroy the batch before them), graph_steps 1..1024.
 *   step:   every member must be ready to step and have unit_check_every = 0
 *           (RTDM_E_UNSUPPORTED otherwise: the check needs the host between
 *           steps).  Returns before the device finishes.  Errors are reported
 *           by rtdm_batch_last_error, not by the members' rtdm_last_error. */
typedef struct rtdm_batch rtdm_batch;
int rtdm_batch_create(rtdm_batch **out, rtdm_ctx *const *ctxs, int n_ctx, int graph_steps);
int rtdm_batch_step(rtdm_batch *batch, double dt, int64_t n_steps, void *hip_stream);
const char *rtdm_batch_last_error(const rtdm_batch *batch);
int rtdm_batch_destroy(rtdm_batch *batch);

/* Observables of the current K: out[0..2] dipole P = -sum_i (r_i - r_c) q_i
 * (Sec. II.B, Mulliken charges q_i = Re sum_j tr(K_ij S_ji), r_c the centroid),
 * out[3] Tr(K S) (Sec. IV), out[4] ||K'-K'^dagger||_F/||K'||_F of the last
 * step's product before Hermitisation, out[5] relative unitarity error
 * ||P_P(U^dagger P_P(S U)) - S||_F / ||S||_F of the current U (Eq. s_unit,
 * computed now).  RTDM_E_NUMERIC if any of out[0..4] is not finite.
 * Synchronises. */
int rtdm_observables(rtdm_ctx *ctx, double out[6], void *hip_stream);

/* Copy the trace recorded since the last kick: row s (s = 0..rows-1) holds
 * t, Px, Py, Pz, Tr(KS), herm_err, unit_err (NaN unless measured at that
 * step) after step s+1.  out has room for max_rows rows of 7 doubles.
 * Synchronises the device. */
int rtdm_dipole_trace(rtdm_ctx *ctx, double *out, int64_t max_rows, int64_t *rows);

/* Unitarity of the current U (Sec. IV, Eq. s_unit, read in the non-orthogonal
 * metric): out[0] = ||D||_F/||S||_F, out[1] = mean |D_ab|, out[2] = max |D_ab|
 * with D = P_P(U^dagger P_P(S U)) - S over R_P's pattern.  Synchronises. */
int rtdm_unitarity(rtdm_ctx *ctx, double out[3], void *hip_stream);

/* Ground-state density matrix of H0 (the state before the kick; Sec. II.A:
 * K S K = K, Tr(K S) = n_occ) by trace-correcting purification (Niklasson,
 * 2002) with truncation, into slot K:
 *   A = P_P(X H0) with X ~ S^-1 (rtdm_build_inverse first);
 *   Z_0 = (hi I - A) / (hi - lo), [lo, hi] from the Gershgorin row discs of A;
 *   per iteration Z^2 = P_P(Z Z); stop when |Tr Z - Tr Z^2| <= tol n_occ, or
 *   when that measure, already below 1e-4 n_occ, stops falling; otherwise
 *   Z <- Z^2 if Tr Z > n_occ, else Z <- 2 Z - Z^2;
 *   K = P_K(Z X), then K <- (K + K^T) / 2.
 * iters, idempotency (the last |Tr Z - Tr Z^2|) and branches (bit k set:
 * iteration k took 2 Z - Z^2) may be NULL.  RTDM_E_NOCONV after max_iter
 * iterations.  Resets the trace and the reference charges like a K upload.
 * Synchronises (two scalars per iteration). */
int rtdm_ground_state(rtdm_ctx *ctx, double n_occ, double tol, int max_iter, void *hip_stream, int *iters,
                      double *idempotency, uint64_t *branches);

/* ---- checkpoint and resume (for long runs split over processes) ----
 * The propagation state beside the matrices: state[0] the time since the
 * kick, state[1] the step count since the kick, then the Mulliken charges
 * q(t), q(t - dt) and q_ref (n_atoms each): 2 + 3 n_atoms doubles (host).
 * Resume = upload S, H0, K (rtdm_download of K at the checkpoint), build or
 * upload the inverse, rtdm_set_state: the following steps then repeat the
 * uninterrupted run bit for bit.  rtdm_set_state starts a new trace.  Both
 * synchronise. */
int rtdm_get_state(rtdm_ctx *ctx, double *state, int64_t n, void *hip_stream);
int rtdm_set_state(rtdm_ctx *ctx, const double *state, int64_t n, void *hip_stream);

/* ---- caller-owned device memory ----
 * Bytes of device memory that hold every buffer of the context now (256-byte
 * aligned), plus a reserve of 64 MiB for the temporaries of later calls and
 * the growth of the observable trace.  Call after set-up (rtdm_set_ranges
 * and the uploads). */
int rtdm_workspace_size(rtdm_ctx *ctx, size_t *bytes);
/* Move every device buffer of the context into the caller's region
 * [ptr, ptr + bytes) (device memory of the context's device, 256-byte
 * aligned, e.g. a torch.empty(bytes, dtype=uint8) tensor) and free the
 * library's own allocations; later allocations of the context are slices of
 * the region (RTDM_E_OOM when it is exhausted).  The region stays owned by
 * the caller and must outlive the context.  Afterwards the geometry and
 * ranges are fixed (RTDM_E_STATE); a captured step graph is rebuilt.  Binding
 * twice is RTDM_E_STATE.  Synchronises the device. */
int rtdm_bind_workspace(rtdm_ctx *ctx, void *ptr, size_t bytes);
/* Device memory from the caller's allocator (e.g. PyTorch's caching
 * allocator): from now on every buffer of the context is alloc_fn(bytes,
 * user) (NULL means out of memory: RTDM_E_OOM; 256-byte alignment required)
 * and is given back with free_fn(ptr, user) when the context releases it
 * (set-up calls, growth of the observable trace, temporaries of calls such as
 * rtdm_multiply, destroy), after a device synchronisation, so that the
 * allocator may reuse it at once on any stream.  The buffers allocated so
 * far move into such allocations.  Once per context (RTDM_E_STATE after that
 * or while a workspace is bound); free_fn must stay callable until
 * rtdm_destroy returns.  Called from the thread of the API call that
 * allocates.  Synchronises the device. */
int rtdm_set_allocator(rtdm_ctx *ctx, void *(*alloc_fn)(size_t bytes, void *user),
                       void (*free_fn)(void *ptr, void *user), void *user);
/* Move every device buffer of the context out of the bound region into
 * allocations of the library's own (the region may be freed afterwards), so
 * that the geometry and ranges can be set again, e.g. to load another system
 * and bind a region of its size (the caller's allocator's, if one is set).  A captured step graph is rebuilt.
 * RTDM_E_STATE without a bound workspace; RTDM_E_OOM (the context stays bound
 * as it was) when the allocations fail.  Synchronises the device. */
int rtdm_unbind_workspace(rtdm_ctx *ctx);
/* Room in the observable trace for `rows` rows in all (every kick set and
 * group), so that steps up to that count allocate nothing; rtdm_step grows
 * the trace itself (from the bound workspace, if any) when a call needs more.
 * The default after set-up is 1,024 rows. */
int rtdm_reserve_trace(rtdm_ctx *ctx, int64_t rows);

/* External field of Gaussian time profile (Sec. II.B, linear response):
 * E(t) = E0 exp(-(t - t0)^2 / (2 sigma^2)) enters H(t) as the electrons'
 * energy E(t) . (r - r_c) (external potential -E . r, electron charge -1),
 * in the position model <i|r|j> = (r_i + r_j)/2 S_ij on R_HS, r_c the
 * centroid of the atom's group.  Time t counts from the last kick.  E0 = 0
 * removes the field.  sigma > 0.  Host arguments, no device work. */
int rtdm_set_field(rtdm_ctx *ctx, const double E0[3], double t0, double sigma);

/* Damped transform of the trace since the last kick (Sec. II.B):
 * F[f](w) = sum_{k=0}^{n} f(t_k) exp((i w - gamma) t_k) dt over t_k = k dt,
 * with the induced dipole P(t_k) - P0 (zero at k = 0).  alpha_jj(w) =
 * F[P_j - P0_j] / F[E_j]: with kappa non-NULL the trace followed the kick
 * exp(i kappa . r), whose field transform is -kappa_j; else the field of
 * rtdm_set_field, sampled at t_k.  group < 0 uses the whole-system trace,
 * group >= 0 that group's trace.  omega[n_omega] (host).  alpha receives
 * [n_omega][3][2] (re, im; NaN where F[E_j] = 0), strength (may be NULL)
 * [n_omega] S(w) = (2 w / pi) Im(sum_j alpha_jj / 3) over the j with a
 * field.  Synchronises. */
int rtdm_spectrum(rtdm_ctx *ctx, int64_t group, const double P0[3], const double *kappa, double gamma,
                  int64_t n_omega, const double *omega, double *alpha, double *strength, void *hip_stream);

/* ---- batches of independent systems ----
 * A batch is one geometry whose atoms fall into contiguous groups placed so
 * that no pair of atoms of different groups is within any range: every
 * matrix is then block-diagonal over groups and every product launch serves
 * all groups.  group_ptr[g] .. group_ptr[g+1]-1 are the atoms of group g
 * (group_ptr[0] = 0, group_ptr[n_groups] = n_atoms).  With more than one
 * group rtdm_step also records per-group observables.  Call after
 * rtdm_set_ranges; RTDM_E_ARG if a kept pair crosses groups. */
int rtdm_set_groups(rtdm_ctx *ctx, int64_t n_groups, const int64_t *group_ptr);
/* K_ij <- exp(i kappa_g . (r_i - r_j)) K_ij with kappa_g = kappa[3g..3g+2]
 * the kick of the group of atoms i and j; otherwise as rtdm_apply_kick. */
int rtdm_apply_kick_groups(rtdm_ctx *ctx, const double *kappa, void *hip_stream);
/* Kick sets (opt.n_kicks > 1, Sec. II.B: the polarisability needs a kick along
 * each axis).  Every set holds its own K (all start from the uploaded K) and
 * shares S, H, X and the step's propagator U, so a step builds U once and
 * updates every K with it.  rtdm_apply_kicks applies kick k (kappa[3k ..
 * 3k+2], bohr^-1, the atom-centred phase of rtdm_apply_kick) to set k, in
 * every group alike; rtdm_apply_kick and rtdm_apply_kick_groups apply their
 * kicks to every set.  rtdm_select_kick chooses the set that rtdm_download
 * (of K), rtdm_observables, rtdm_dipole_trace, rtdm_group_trace,
 * rtdm_spectrum and rtdm_get_state report (default 0); rtdm_set_state
 * needs n_kicks = 1. */
int rtdm_apply_kicks(rtdm_ctx *ctx, const double *kappa, void *hip_stream);
int rtdm_select_kick(rtdm_ctx *ctx, int k);

/* Per-group trace since the last kick: out[(s * n_groups + g) * 4 + 0..3] =
 * (Px, Py, Pz, Tr(KS)) of group g after step s+1, the dipole taken about the
 * group's centroid.  Synchronises. */
int rtdm_group_trace(rtdm_ctx *ctx, double *out, int64_t max_rows, int64_t *rows);

/* Time candidate launch shapes of the step's block products (workgroups of
 * 4, 8 or 16 waves for the single-output kernels; output tiles of 64, 256 or
 * 1024 atom rows) on the current matrices and keep the fastest; b = 13 only
 * (other block sizes have one shape).  Overwrites W and the Taylor-term work buffers.  *wpb, *row_tile
 * (may be NULL) receive the choice.  Synchronises. */
int rtdm_autotune(rtdm_ctx *ctx, void *hip_stream, int *wpb, int *row_tile);

/* Outcome of the last rtdm_build_inverse: iterations summed over the start
 * and, if taken, the block-Jacobi fallback; fell_back = 1 if the fallback ran.
 * Either pointer may be NULL. */
int rtdm_inverse_info(rtdm_ctx *ctx, int *iters_total, int *fell_back);

/* ---- learned starting guess (a two-layer perceptron, hidden width 128) ----
 * The network maps the descriptor of an atom-pair block (i, j) of S's range,
 *   d = [(r_i - r_j)/R_HS (3), |r_i - r_j|/R_HS, S_ij (b*b, row-major)]  (4 + b*b floats),
 * to a correction y (b*b floats) of the first-order start 2 delta_ij I - S_ij.
 * Parameters (FP32 master copy, this order): W1 (128 x in, row-major), b1
 * (128), W2 (out x 128), b2 (out); the forward pass uses FP16 copies of W1 and
 * W2 with FP32 accumulation: y = W2 tanh(W1 d + b1) + b2.  Training minimises
 * the mean squared error over the collected samples with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  The network's size follows the
 * geometry's b; it survives rtdm_set_ranges, not rtdm_set_geometry with a
 * different b.  All calls synchronise. */
int rtdm_mlp_params(rtdm_ctx *ctx, int64_t *n_params, int *in, int *hidden, int *out);
/* Initialise the weights (uniform +-1/sqrt(fan_in), second layer scaled by 0.1,
 * zero biases) from `seed`, reset Adam's state. */
int rtdm_mlp_init(rtdm_ctx *ctx, uint64_t seed);
/* Set / read the FP32 master weights (host arrays of n_params floats). */
int rtdm_mlp_set_weights(rtdm_ctx *ctx, const float *w, int64_t n);
int rtdm_mlp_get_weights(rtdm_ctx *ctx, float *w, int64_t n);
/* Append training samples from the current S and the converged X: up to
 * max_samples blocks of S's range chosen by a seeded shuffle; the target is
 * X_ij - (2 delta_ij I - S_ij).  *total receives the dataset size. */
int rtdm_mlp_collect(rtdm_ctx *ctx, int64_t max_samples, uint64_t seed, int64_t *total);
int rtdm_mlp_clear(rtdm_ctx *ctx);
/* Adam over `epochs` passes of the dataset in seeded random mini-batches of
 * `batch` samples at learning rate lr; *loss receives the mean squared error
 * of the last epoch (per output element). */
int rtdm_mlp_train(rtdm_ctx *ctx, int epochs, int batch, double lr, uint64_t seed, double *loss);
/* Test entries: the loss (mean squared error per output element) and its
 * gradient w.r.t. the master weights for n host samples (desc n x in, target
 * n x out), without updating; and the forward pass for n host descriptors. */
int rtdm_mlp_loss_grad(rtdm_ctx *ctx, int64_t n, const float *desc, const float *target, double *loss,
                       float *grad);
/* Test entry: one Adam step (Kingma and Ba 2015; beta1 0.9, beta2 0.999,
 * eps 1e-8, the constants of rtdm_mlp_train) on the gradient of the loss of
 * n host samples (desc n x in, target n x out, copied) at learning rate lr;
 * the step counter and moments continue from the previous steps and restart
 * at rtdm_mlp_init / rtdm_mlp_set_weights.  *loss receives the loss before
 * the step.  Synchronises. */
int rtdm_mlp_step(rtdm_ctx *ctx, int64_t n, const float *desc, const float *target, double lr, double *loss);
int rtdm_mlp_predict(rtdm_ctx *ctx, int64_t n, const float *desc, float *y);

/* Truncation error of the inverse (Sec. V.A, the paper's measure of the
 * S^-1 truncation): D = P_P(X S) - I over R_P's pattern; out[0] = mean |D_ab|
 * over the pattern's elements, out[1] = max |D_ab|, out[2] = ||D||_F.
 * Needs a built or uploaded X.  Synchronises. */
int rtdm_inverse_error(rtdm_ctx *ctx, double out[3], void *hip_stream);

/* Test entry: C = P_C(alpha op(A) op(B)) on the slots' patterns, where op is
 * the identity (0) or the conjugate transpose (1).  The (range(A), range(B),
 * range(C), op_a, op_b) combination must be one of RTDM_PROD_* (else
 * RTDM_E_UNSUPPORTED).  C becomes complex if A, B or alpha is.  At b = 13
 * in FP64 or FP32 the step kinds (X H, A tau, U K, W U^dagger) with a real
 * alpha run the step's kernels and layouts; the call then synchronises. */
int rtdm_multiply(rtdm_ctx *ctx, rtdm_mat C, rtdm_mat A, rtdm_mat B, int op_a, int op_b,
                  double alpha_re, double alpha_im, void *hip_stream);

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * rtdm_multiply with the same arguments and results, whose b = 13
 * column-major operand copies live in a static device array of
 * 128 MiB per GPU (held from the library's first use on that GPU until the
 * process ends) instead of fresh allocations.  It calls no hipMalloc or
 * hipFree and does not synchronise (it is asynchronous on hip_stream).
 * Errors: RTDM_E_ARG when the copies (the planes of A, of B if op_b = 1, of
 * C for the U K kind) exceed 128 MiB; RTDM_E_STATE when the product kind has
 * no schedule yet (the five step kinds are scheduled by rtdm_set_ranges;
 * another kind needs one rtdm_multiply first).  Every call on a GPU, from any
 * context, shares that GPU's array and overwrites it: calls that overlap on
 * one GPU (two streams, two host threads) race. */
int rtdm_multiply_noalloc(rtdm_ctx *ctx, rtdm_mat C, rtdm_mat A, rtdm_mat B, int op_a, int op_b,
                          double alpha_re, double alpha_im, void *hip_stream);

/* Symbolic sizes of a product: number of output blocks and of (i,k,j) block
 * triples that survive all three cut-offs (the algorithmic unit of work,
 * 2 b^3 flops per real block product). */
int rtdm_schedule_stats(rtdm_ctx *ctx, rtdm_prod prod, int64_t *outputs, int64_t *triples);

/* Per-launch HIP-event timing of the block-product kernels, for measurement.
 * enable = 1 starts recording (and clears earlier records), 0 stops. */
int rtdm_timing(rtdm_ctx *ctx, int enable);

/* Totals of the recorded product launches of one kind: launches, summed
 * kernel milliseconds, summed algorithmic flops.  Synchronises. */
int rtdm_timing_stats(rtdm_ctx *ctx, rtdm_prod prod, int64_t *launches, double *total_ms,
                      double *flops);

/* Message of the last failing call on ctx ("" if none; a static message for
 * a NULL ctx). */
const char *rtdm_last_error(const rtdm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* RTDM_H */

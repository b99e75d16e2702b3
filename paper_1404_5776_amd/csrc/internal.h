// Internal declarations of the rtdm library (not part of the C ABI).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <unordered_set>
#include <utility>

#include "rtdm.h"

namespace rtdm {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define RT_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::rtdm::Error(RTDM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define RT_CHECK(cond, code, msg)                         \
    do {                                                  \
        if (!(cond)) throw ::rtdm::Error((code), (msg));  \
    } while (0)

// Device memory of one context.  Every buffer the context allocates is
// registered here.  A buffer owns an allocation of the caller's allocator
// (rtdm_set_allocator) or, without one, a hipMalloc allocation; once the
// caller binds a workspace (rtdm_bind_workspace) every registered buffer is
// moved into it and later allocations are 256-byte aligned slices of it,
// taken in order (a released slice is reused only when it is the last one).
struct DBufBase;
struct DevMem {
    std::unordered_set<DBufBase *> bufs;
    char *base = nullptr;
    size_t cap = 0, used = 0;
    void *(*ext_alloc)(size_t bytes, void *user) = nullptr;   // the caller's allocator, if set
    void (*ext_free)(void *ptr, void *user) = nullptr;
    void *ext_user = nullptr;
};
// The context of the API call in progress on this thread (null outside calls).
extern thread_local DevMem *g_devmem;

struct DBufBase {
    DevMem *mem = nullptr;   // registry the buffer belongs to (null: unregistered)
    bool in_ws = false;      // the memory is a slice of a bound workspace
    bool ext = false;        // the memory came from the caller's allocator
    size_t nbytes = 0;
    virtual void *raw() const = 0;
    virtual void set_raw(void *p) = 0;
    virtual ~DBufBase() = default;
};
void *devmem_alloc(DBufBase *b, size_t bytes);
void devmem_free(DBufBase *b, void *p);
void devmem_moved(DBufBase *from, DBufBase *to);
inline size_t devmem_align(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

// Owning device buffer.
template <class T>
struct DBuf : DBufBase {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept { take(o); }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); take(o); }
        return *this;
    }
    ~DBuf() override { release(); }
    void alloc(size_t count) {
        if (count == n && p) return;
        release();
        if (count == 0) return;
        p = static_cast<T *>(devmem_alloc(this, count * sizeof(T)));
        n = count;
    }
    void release() {
        if (p) devmem_free(this, p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    void *raw() const override { return p; }
    void set_raw(void *q) override { p = static_cast<T *>(q); }

private:
    void take(DBuf &o) noexcept {
        p = o.p;
        n = o.n;
        mem = o.mem;
        in_ws = o.in_ws;
        ext = o.ext;
        nbytes = o.nbytes;
        devmem_moved(&o, this);
        o.p = nullptr;
        o.n = 0;
        o.mem = nullptr;
        o.nbytes = 0;
        o.in_ws = false;
    }
};

// ---------------------------------------------------------------- kernels

// Symbolic phase of C = P_C(op(A) op(B)): per output block (i, j) of C, the
// ascending k with op(A)_ik and op(B)_kj stored.
void launch_sym_count(hipStream_t s, int64_t nout, const int32_t *c_rowof, const int32_t *c_col,
                      const int64_t *a_ptr, const int32_t *a_col, const int64_t *b_ptr,
                      const int32_t *b_col, int64_t *cnt);
void launch_sym_fill(hipStream_t s, int64_t nout, const int32_t *c_rowof, const int32_t *c_col,
                     const int64_t *a_ptr, const int32_t *a_col, const int32_t *a_trans,
                     const int64_t *b_ptr, const int32_t *b_col, const int32_t *b_trans, int op_a,
                     int op_b, const int64_t *off, int2 *trip);

struct SpgemmArgs {
    int64_t nout = 0;
    const int64_t *off = nullptr;   // [nout+1] triple offsets
    const int2 *trip = nullptr;     // (block of op(A), block of op(B)) per triple
    const double *ar = nullptr, *ai = nullptr;   // ai null: A real
    const double *br = nullptr, *bi = nullptr;   // bi null: B real
    double *cr = nullptr, *ci = nullptr;         // ci null: C real
    int b = 0;
    int op_a = 0, op_b = 0;          // 1: conjugate transpose
    double alpha_re = 1.0, alpha_im = 0.0;
    int precision = RTDM_PREC_FP64;  // arithmetic of the block products
    const double *zero = nullptr;    // 256 zero doubles (operand of lanes without data)
    const int32_t *order = nullptr;  // processing order of the output blocks (null: storage order)
    int wpb = 16;                    // waves per workgroup of the step kernels (4, 8, 16)
    // FP16 split products: [8k .. 8k+3] the reduction of operand k's (A: 0,
    // B: 1) real plane, [8k+4 .. 8k+7] of its imaginary plane (zeros if
    // real); the last slot of each holds max |x|.
    const double *maxabs = nullptr;
    // Row runs of the b = 13 step products (launch_spgemm_cm when nch > 0):
    // run c covers the outputs ch_out[c*nj .. c*nj+nj-1] (-1: none) of one row
    // i of C; its entries ch_off[c] .. ch_off[c+1]-1 are the contraction
    // indices k used by any of them, entry e naming op(A)_ik (ch_a[e]) and
    // op(B)_kj of each output (ch_b[e*nj + t], -1 where that output has no
    // triple with this k).  ch_order: processing order of the runs.
    int nj = 0;
    int64_t nch = 0;
    const int64_t *ch_off = nullptr;
    const int32_t *ch_a = nullptr, *ch_b = nullptr, *ch_out = nullptr, *ch_order = nullptr;
    const int32_t *ch_seg = nullptr;   // runs of 2: per run the entries feeding both outputs, then only the first
};
void launch_spgemm(hipStream_t s, const SpgemmArgs &a);
// Row runs, op(A) = A: entry counts per run, then the entries (SpgemmArgs::ch_*;
// inter4: the b = 4 kernel's slot order) and the output map of every run.
// seg (count pass, runs of 2, nullable): per run the sizes of the segments
// of entries feeding both outputs and only the first; `segmented` (fill
// pass): store the entries in that segment order.
void launch_run_count(hipStream_t s, int64_t nch, const int32_t *run_row, const int64_t *run_p0, const int64_t *c_ptr,
                      const int32_t *c_col, const int64_t *a_ptr, const int32_t *a_col, const int64_t *b_ptr,
                      const int32_t *b_col, int nj, int64_t *cnt, int32_t *seg);
void launch_run_fill(hipStream_t s, int64_t nch, const int32_t *run_row, const int64_t *run_p0, const int64_t *c_ptr,
                     const int32_t *c_col, const int64_t *a_ptr, const int32_t *a_col, const int64_t *b_ptr,
                     const int32_t *b_col, const int32_t *b_trans, int op_b, int nj, int inter4, const int64_t *off,
                     int32_t *ea, int32_t *eb, int32_t *rout, int segmented);
// Same product with the left operand given as column-major blocks, the right
// operand's op(B)[m][r] at m*B + r (conj_b: conjugated) and the output written
// column-major if out_col_major.  b = 13, FP64.
void launch_spgemm_cm(hipStream_t s, const SpgemmArgs &a, int conj_b, int out_col_major);
// Split-precision (BF16X3 / FP16X2) step product of real operands: column-
// major left operand, row-major right operand, row-major FP64 output.
void launch_spgemm_cm_split(hipStream_t s, const SpgemmArgs &a);
// Real FP32 step product: a32 column-major left operand, b32 row-major right
// operand, c32 = alpha * P_C(A B) row-major FP32 (b = 13).
void launch_spgemm_r32(hipStream_t s, const SpgemmArgs &a, const float *a32, const float *b32, float *c32,
                       const float *zero32);
// out = (float)in, optionally transposing every b x b block.
void launch_to_f32(hipStream_t s, int64_t nblocks, int b, int transpose, const double *in, float *out);
// b = 4 blocks as BF16 hi / lo parts, 32 values per block (its 16 hi parts,
// then its 16 lo parts; transpose: each block stored transposed)
void launch_to_bf16x2(hipStream_t s, int64_t nblocks, int transpose, const double *in, short *out);
// BF16x3 Taylor term at b = 4 over row runs of 16 (a.ch_*, alpha a.alpha_re) from split
// operands: u += u_sign * tau, and tau stored split and transposed in c16 (if set)
void launch_spgemm_r16(hipStream_t s, const SpgemmArgs &a, const short *a16, const short *b16, short *c16,
                       double *u, double u_sign);
// y += a * (double)x
void launch_axpy_f32(hipStream_t s, int64_t n, double a, const float *x, double *y);
// out[p] = in[p]^T for every b x b block (nblocks blocks).
void launch_transpose_blocks(hipStream_t s, int64_t nblocks, int b, const double *in, double *out);
// out_ji = in_ij^dagger over a pattern (trans: the transpose map of the pattern)
void launch_conj_transpose(hipStream_t s, int64_t nnzb, int b, const int32_t *trans, const double *in_re,
                           const double *in_im, double *out_re, double *out_im);
// True when a b = 4 product over nch runs of 16 outputs takes the split form
// (one workgroup per run: small systems, whose runs are too few to fill the chip).
bool b4_split_form(int64_t nch);

// out = a*x + c*y elementwise (y may be null: out = a*x).
void launch_axpby(hipStream_t s, int64_t n, double a, const double *x, double c, const double *y,
                  double *out);
// m[diag blocks] += val * I.
void launch_add_identity(hipStream_t s, int64_t n_atoms, int b, const int32_t *diag, double val,
                         double *m);
// K_ij *= exp(i kappa.(r_i - r_j)).
void launch_kick(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof, const int32_t *col,
                 const double *xyz, double kx, double ky, double kz, double *kr, double *ki);
// K = (Kn + Kn^H)/2 with partial sums of ||Kn - Kn^H||^2 and ||Kn||^2.
void launch_hermitize(hipStream_t s, int64_t nnzb, int b, const int32_t *trans, const double *knr,
                      const double *kni, double *kr, double *ki, double *partials);
// q_i = Re sum_j tr(K_ij S_ji).
void launch_mulliken(hipStream_t s, int64_t n_atoms, int b, const int64_t *s_ptr,
                     const int32_t *s_trans, const int32_t *s_to_k, const double *sv,
                     const double *kr, double *q);
// H[diag] += gain*(q_a + theta (q_x - q_y) - q_ref) on the diagonal elements.
void launch_add_scalar(hipStream_t s, double *x, double v);
void launch_a_onsite(hipStream_t s, int64_t nnzb, int b, const int32_t *col, const int32_t *nbf, double gain,
                     const double *q_a, double theta, const double *q_x, const double *q_y, const double *q_ref,
                     const double *a0, const double *x, double *a);
void launch_onsite_shift(hipStream_t s, int64_t n_atoms, int b, const int32_t *diag, const int32_t *nbf, double gain,
                         const double *q_a, double theta, const double *q_x, const double *q_y,
                         const double *q_ref, double *h);
void launch_field(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof, const int32_t *col,
                  const double *xyz, const int32_t *group, const double *centre, const double *sv,
                  const double E0[3], double t0, double sigma, const int64_t *st, const double *tt,
                  double theta, double *h);
void launch_spectrum(hipStream_t s, int64_t n_omega, const double *omega, double gamma, double dt, int64_t n,
                     const double *trace, int64_t stride, int64_t off, const double P0[3], int kick,
                     const double E0[3], double t0, double sigma, double *alpha, double *strength);
// Observable row: t, P(3), Tr(KS), herm_err from (partials -> sums), unit_err = NaN.
// centre: the atoms' centroid (3 doubles, computed on the host with an exactly rounded sum).
void launch_observables(hipStream_t s, int64_t n_atoms, const double *xyz, const double *centre, const double *q,
                        const double *herm_sums, double t, double *row);
// The same observables written to obs + 8 * st[0] at time tt[0] + (st[1] + 1) * tt[1].
void launch_observables_step(hipStream_t s, int64_t n_atoms, const double *xyz, const double *centre,
                             const double *q, const double *herm_sums, double *obs, int64_t *st, const double *tt);
void launch_step_begin(hipStream_t s, int64_t *st, double *tt, double t0, double dt);
void launch_step_end(hipStream_t s, int64_t *st);
void launch_fill(hipStream_t s, int64_t n, double v, double *out);
void launch_group_obs(hipStream_t s, int64_t n_groups, const int64_t *gptr, const double *xyz, const double *centre,
                      const double *q, const int64_t *st, double *out);
void launch_kick_groups(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof, const int32_t *col,
                        const double *xyz, const int32_t *group, const double *kappa, double *kr, double *ki);
// X_ii = S_ii^{-1} (Gauss-Jordan, partial pivoting); other blocks untouched.
void launch_block_inverse(hipStream_t s, int64_t n_atoms, int b, const int32_t *s_diag,
                          const double *sv, const int32_t *x_diag, double *xv, double *scratch);
// per-atom max absolute row sum of S.
void launch_row_abs_max(hipStream_t s, int64_t n_atoms, int b, const int64_t *s_ptr,
                        const double *sv, double *atom_max);

// Deterministic reductions: partials[G][4] then finish -> out[4].
constexpr int kRedBlocks = 512;
void launch_red_diff2(hipStream_t s, int64_t n, const double *x, const double *y, double *partials);
void launch_red_unitarity(hipStream_t s, int64_t nnzb_p, int b, const int32_t *p_to_hs,
                          const double *sv, const double *zr, const double *zi, double *partials);
// sums of |v - I| over a pattern's elements: [0] sum |d|^2, [1] sum |d|, [3] max |d|
void launch_red_minus_identity(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof,
                               const int32_t *col, const double *v, double *partials);
void launch_red_sumsq(hipStream_t s, int64_t n, const double *x, double *partials);
void launch_red_trace(hipStream_t s, int64_t n_atoms, int b, const int32_t *diag, const double *v,
                      double *partials);
void launch_gershgorin(hipStream_t s, int64_t n_atoms, int b, const int64_t *rowptr, const int32_t *diag,
                       const double *v, double *lohi);
void launch_red_max(hipStream_t s, int64_t n, const double *x, double *partials);
void launch_red_finish(hipStream_t s, const double *partials, double *out);
// unit-row update: row[6] = sqrt(sums[0] / s2)
void launch_unit_to_row(hipStream_t s, const double *unit_sums, const double *s_norm2, double *row);

// interleave / split complex128
void launch_split(hipStream_t s, int64_t n, const double *inter, double *re, double *im);
void launch_interleave(hipStream_t s, int64_t n, const double *re, const double *im, double *inter);

// ---------------------------------------------------------------- static scratch
// Size of the file-scope device array behind rtdm_multiply_noalloc (per GPU).
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
// Device address of that array on `device`, which must be current; looked up
// (hipGetSymbolAddress) on the first call per device.
double *static_scratch(int device);

// ---------------------------------------------------------------- learned start
constexpr int kMlpHidden = 128;
void launch_mlp_desc(hipStream_t s, int64_t n, int b, const int32_t *blk, const int32_t *rowof,
                     const int32_t *col, const double *xyz, const double *sv, double inv_r, float *desc);
void launch_mlp_target(hipStream_t s, int64_t n, int b, const int32_t *blk, const int32_t *x_of,
                       const int32_t *rowof, const int32_t *col, const double *sv, const double *xv,
                       float *tgt);
void launch_mlp_forward(hipStream_t s, int64_t n, int in, int out, const int32_t *idx, const float *x,
                        const __half *w1, const float *b1, const __half *w2, const float *b2, float *hid,
                        float *y);
void launch_mlp_delta(hipStream_t s, int64_t n, int out, const int32_t *idx, const float *tgt, const float *y,
                      const float *hid, const __half *w2, float *dy, float *dh, float *sqerr);
void launch_mlp_grad(hipStream_t s, int64_t n, int in, int out, const int32_t *idx, const float *x,
                     const float *hid, const float *dy, const float *dh, float *grad);
void launch_adam(hipStream_t s, int64_t np, int64_t nw1, int64_t nb1, int64_t nw2, const float *grad, float *w,
                 float *m, float *v, float lr, double beta1, double beta2, float eps, int step, __half *w1h,
                 __half *w2h);
void launch_to_half(hipStream_t s, int64_t n, const float *x, __half *y);
void launch_mlp_apply(hipStream_t s, int64_t n, int b, const int32_t *blk, const int32_t *x_of,
                      const int32_t *rowof, const int32_t *col, const double *sv, const float *y, double *xv);
void launch_sum_f32(hipStream_t s, int64_t n, const float *x, double *out);

}  // namespace rtdm

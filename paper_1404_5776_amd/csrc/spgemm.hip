// Truncated block-sparse products C = P_C(alpha op(A) op(B)) on gfx950.
//
// Every matrix is stored in atom-pair blocks on a spatial cut-off pattern
// (Sec. II.A); a product keeps only the output blocks inside C's cut-off
// (Sec. V.A truncates S^-1 and S^-1 H, and every product of a step is
// truncated the same way).
//
// Symbolic phase (once per pattern triple): for output block (i, j) the k with
// op(A)_ik and op(B)_kj stored are the common entries of row i of A's pattern
// and row j of B's pattern (cut-off patterns are symmetric, so "k in row j"
// is "(k, j) kept").  One thread per output block merges the two ascending
// lists; a count pass sizes the triple list, a fill pass writes
// (block index of op(A)_ik, block index of op(B)_kj), ascending in k.
//
// Numeric phase: one 64-lane wave per output block accumulates its triples
// with the FP64 matrix cores (v_mfma_f64_16x16x4_f64): a b x b block (b <= 16)
// sits in one 16 x 16 tile and the contraction runs in steps of 4.  Complex
// operands are split into real and imaginary planes, so a complex block
// product is four real tile products (re*re, im*im, re*im, im*re) sharing the
// operand loads; a real operand skips the products it does not need.
#include "internal.h"

namespace rtdm {

typedef double d4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- symbolic

__global__ void k_sym_count(int64_t nout, const int32_t *__restrict__ c_rowof,
                            const int32_t *__restrict__ c_col, const int64_t *__restrict__ a_ptr,
                            const int32_t *__restrict__ a_col, const int64_t *__restrict__ b_ptr,
                            const int32_t *__restrict__ b_col, int64_t *__restrict__ cnt)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nout) return;
    const int i = c_rowof[c], j = c_col[c];
    int64_t pa = a_ptr[i], ea = a_ptr[i + 1], pb = b_ptr[j], eb = b_ptr[j + 1];
    int64_t n = 0;
    while (pa < ea && pb < eb) {
        const int ka = a_col[pa], kb = b_col[pb];
        n += (ka == kb);
        pa += (ka <= kb);
        pb += (kb <= ka);
    }
    cnt[c] = n;
}

__global__ void k_sym_fill(int64_t nout, const int32_t *__restrict__ c_rowof,
                           const int32_t *__restrict__ c_col, const int64_t *__restrict__ a_ptr,
                           const int32_t *__restrict__ a_col, const int32_t *__restrict__ a_trans,
                           const int64_t *__restrict__ b_ptr, const int32_t *__restrict__ b_col,
                           const int32_t *__restrict__ b_trans, int op_a, int op_b,
                           const int64_t *__restrict__ off, int2 *__restrict__ trip)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nout) return;
    const int i = c_rowof[c], j = c_col[c];
    int64_t pa = a_ptr[i], ea = a_ptr[i + 1], pb = b_ptr[j], eb = b_ptr[j + 1];
    int64_t o = off[c];
    while (pa < ea && pb < eb) {
        const int ka = a_col[pa], kb = b_col[pb];
        if (ka == kb) {
            // op(A)_ik: block (i,k) = pa, or (k,i) = trans[pa] for the conjugate transpose.
            // op(B)_kj: block (k,j) = trans[pb] (pb is (j,k)), or (j,k) = pb for the conjugate transpose.
            const int ia = op_a ? a_trans[pa] : (int)pa;
            const int ib = op_b ? (int)pb : b_trans[pb];
            trip[o++] = make_int2(ia, ib);
        }
        pa += (ka <= kb);
        pb += (kb <= ka);
    }
}

void launch_sym_count(hipStream_t s, int64_t nout, const int32_t *c_rowof, const int32_t *c_col,
                      const int64_t *a_ptr, const int32_t *a_col, const int64_t *b_ptr,
                      const int32_t *b_col, int64_t *cnt)
{
    if (nout == 0) return;
    const int T = 256;
    hipLaunchKernelGGL(k_sym_count, dim3((unsigned)((nout + T - 1) / T)), dim3(T), 0, s, nout,
                       c_rowof, c_col, a_ptr, a_col, b_ptr, b_col, cnt);
    RT_HIP(hipGetLastError());
}

void launch_sym_fill(hipStream_t s, int64_t nout, const int32_t *c_rowof, const int32_t *c_col,
                     const int64_t *a_ptr, const int32_t *a_col, const int32_t *a_trans,
                     const int64_t *b_ptr, const int32_t *b_col, const int32_t *b_trans, int op_a,
                     int op_b, const int64_t *off, int2 *trip)
{
    if (nout == 0) return;
    const int T = 256;
    hipLaunchKernelGGL(k_sym_fill, dim3((unsigned)((nout + T - 1) / T)), dim3(T), 0, s, nout,
                       c_rowof, c_col, a_ptr, a_col, a_trans, b_ptr, b_col, b_trans, op_a, op_b,
                       off, trip);
    RT_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- numeric

// MFMA 16x16x4 f64 operand layout (wave of 64 lanes, lane = 16*q + r):
//   A operand: lane supplies A[r][q]   (row r of the 16x4 slice, column q)
//   B operand: lane supplies B[q][r]   (row q of the 4x16 slice, column r)
//   D (4 doubles per lane): element e of lane is D[4*q + e][r]
template <bool AC, bool BC, int OPA, int OPB>
__global__ __launch_bounds__(256) void k_spgemm16(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, int b,
    double alr, double ali)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nout) return;                     // uniform across the wave
    const int bb = b * b;
    const int r = lane & 15, q = lane >> 4;
    d4 rr = {0, 0, 0, 0}, ii = {0, 0, 0, 0}, ri = {0, 0, 0, 0}, ir = {0, 0, 0, 0};
    const int64_t t0 = off[c], t1 = off[c + 1];
    for (int64_t t = t0; t < t1; ++t) {
        const int2 ab = trip[t];
        const int64_t abase = (int64_t)ab.x * bb, bbase = (int64_t)ab.y * bb;
        for (int k0 = 0; k0 < b; k0 += 4) {
            const int kk = k0 + q;
            const bool ok = (r < b) && (kk < b);
            const int ia = OPA ? (kk * b + r) : (r * b + kk);   // op(A)[r][kk]
            const int ib = OPB ? (r * b + kk) : (kk * b + r);   // op(B)[kk][r]
            double xar = 0.0, xai = 0.0, xbr = 0.0, xbi = 0.0;
            if (ok) {
                xar = ar[abase + ia];
                xbr = br[bbase + ib];
                if (AC) xai = OPA ? -ai[abase + ia] : ai[abase + ia];
                if (BC) xbi = OPB ? -bi[bbase + ib] : bi[bbase + ib];
            }
            rr = __builtin_amdgcn_mfma_f64_16x16x4f64(xar, xbr, rr, 0, 0, 0);
            if (AC && BC) ii = __builtin_amdgcn_mfma_f64_16x16x4f64(xai, xbi, ii, 0, 0, 0);
            if (BC) ri = __builtin_amdgcn_mfma_f64_16x16x4f64(xar, xbi, ri, 0, 0, 0);
            if (AC) ir = __builtin_amdgcn_mfma_f64_16x16x4f64(xai, xbr, ir, 0, 0, 0);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = 4 * q + e, col = r;
        if (row < b && col < b) {
            const double re = rr[e] - ii[e];
            const double im = ri[e] + ir[e];
            const int64_t o = c * bb + row * b + col;
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

// Compile-time block size B <= 16 with the contraction concatenated across the
// triples of one output block: the kappa-th contraction index is element m of
// triple tt (kappa = B*tt + m), so the 4-wide MFMA steps run over B*ntrip
// indices instead of padding every triple from B to a multiple of 4.  Lane
// (q, r) supplies index kappa = 4*s + q at step s.  The operands of step s+1
// are loaded before the matrix-core work of step s is issued.
template <int B, bool AC, bool BC, int OPA, int OPB>
__global__ __launch_bounds__(256) void k_spgemm_kc(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, double alr,
    double ali)
{
    static_assert(B >= 4 && B <= 16, "k_spgemm_kc needs 4 <= B <= 16");
    constexpr int BB = B * B;
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nout) return;                     // uniform across the wave
    const int r = lane & 15, q = lane >> 4;
    const bool rv = r < B;
    const int64_t t0 = off[c];
    const int nt = (int)(off[c + 1] - t0);
    const int steps = (B * nt + 3) >> 2;
    // per-lane element offsets inside a block for op(A)[r][m] and op(B)[m][r]
    const int oa_r = OPA ? r : r * B;          // + m * (OPA ? B : 1)
    const int ob_r = OPB ? r * B : r;          // + m * (OPB ? 1 : B)
    constexpr int sa = OPA ? B : 1, sb = OPB ? 1 : B;

    int tt = 0, m = q;                         // B >= 4: the first step stays in triple 0
    int2 ab = nt > 0 ? trip[t0] : make_int2(0, 0);
    double xar = 0.0, xai = 0.0, xbr = 0.0, xbi = 0.0;
    auto fetch = [&](double &far, double &fai, double &fbr, double &fbi) {
        far = fai = fbr = fbi = 0.0;
        if (tt < nt && rv) {
            const int64_t pa = (int64_t)ab.x * BB + oa_r + m * sa;
            const int64_t pb = (int64_t)ab.y * BB + ob_r + m * sb;
            far = ar[pa];
            fbr = br[pb];
            if (AC) fai = OPA ? -ai[pa] : ai[pa];
            if (BC) fbi = OPB ? -bi[pb] : bi[pb];
        }
    };
    auto advance = [&]() {
        m += 4;
        if (m >= B) {
            m -= B;
            ++tt;
            if (tt < nt) ab = trip[t0 + tt];
        }
    };
    d4 rr = {0, 0, 0, 0}, ii = {0, 0, 0, 0}, ri = {0, 0, 0, 0}, ir = {0, 0, 0, 0};
    fetch(xar, xai, xbr, xbi);
    for (int s = 0; s < steps; ++s) {
        advance();
        double nar, nai, nbr, nbi;
        fetch(nar, nai, nbr, nbi);
        rr = __builtin_amdgcn_mfma_f64_16x16x4f64(xar, xbr, rr, 0, 0, 0);
        if (AC && BC) ii = __builtin_amdgcn_mfma_f64_16x16x4f64(xai, xbi, ii, 0, 0, 0);
        if (BC) ri = __builtin_amdgcn_mfma_f64_16x16x4f64(xar, xbi, ri, 0, 0, 0);
        if (AC) ir = __builtin_amdgcn_mfma_f64_16x16x4f64(xai, xbr, ir, 0, 0, 0);
        xar = nar;
        xai = nai;
        xbr = nbr;
        xbi = nbi;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = 4 * q + e, col = r;
        if (row < B && col < B) {
            const double re = rr[e] - ii[e];
            const double im = ri[e] + ir[e];
            const int64_t o = c * BB + row * B + col;
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

template <bool AC, bool BC>
static void dispatch_ops(hipStream_t s, const SpgemmArgs &a, dim3 g, dim3 t)
{
#define RT_LAUNCH(OA, OB)                                                                        \
    do {                                                                                         \
        if (a.b == 13)                                                                           \
            hipLaunchKernelGGL((k_spgemm_kc<13, AC, BC, OA, OB>), g, t, 0, s, a.nout, a.off,     \
                               a.trip, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,           \
                               a.alpha_im);                                                      \
        else if (a.b == 16)                                                                      \
            hipLaunchKernelGGL((k_spgemm_kc<16, AC, BC, OA, OB>), g, t, 0, s, a.nout, a.off,     \
                               a.trip, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,           \
                               a.alpha_im);                                                      \
        else                                                                                     \
            hipLaunchKernelGGL((k_spgemm16<AC, BC, OA, OB>), g, t, 0, s, a.nout, a.off, a.trip,  \
                               a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.b, a.alpha_re, a.alpha_im); \
    } while (0)
    if (!a.op_a && !a.op_b) RT_LAUNCH(0, 0);
    else if (a.op_a && !a.op_b) RT_LAUNCH(1, 0);
    else if (!a.op_a && a.op_b) RT_LAUNCH(0, 1);
    else RT_LAUNCH(1, 1);
#undef RT_LAUNCH
}

void launch_spgemm(hipStream_t s, const SpgemmArgs &a)
{
    if (a.nout == 0) return;
    RT_CHECK(a.b >= 1 && a.b <= 16, RTDM_E_UNSUPPORTED, "block size must be 1..16");
    const dim3 g((unsigned)((a.nout + 3) / 4)), t(256);
    const bool ac = a.ai != nullptr, bc = a.bi != nullptr;
    if (ac && bc) dispatch_ops<true, true>(s, a, g, t);
    else if (ac) dispatch_ops<true, false>(s, a, g, t);
    else if (bc) dispatch_ops<false, true>(s, a, g, t);
    else dispatch_ops<false, false>(s, a, g, t);
    RT_HIP(hipGetLastError());
}

}  // namespace rtdm

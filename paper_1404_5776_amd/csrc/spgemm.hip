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
#include <cstdlib>
#include <type_traits>

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

// Row runs (see SpgemmArgs::ch_*): one thread per run of up to nj (<= 16)
// consecutive outputs p0 .. p1-1 of row i of C, op(A) = A.  The thread walks
// row i of A (ascending k) and, in step, the rows j_t of B's pattern (the
// patterns are symmetric, so k in row j_t means block (k, j_t) exists); an
// entry is a k present for at least one output.  Slot of output t in an
// entry: t, or (t % 4) * 4 + t / 4 with `inter4` (the lane order of the b = 4
// kernel, whose lane group g reads outputs g, g + 4, g + 8, g + 12).
constexpr int kMaxRun = 16;
template <bool FILL>
__global__ void k_run_sym(int64_t nch, const int32_t *__restrict__ run_row, const int64_t *__restrict__ run_p0,
                          const int64_t *__restrict__ c_ptr, const int32_t *__restrict__ c_col,
                          const int64_t *__restrict__ a_ptr, const int32_t *__restrict__ a_col,
                          const int64_t *__restrict__ b_ptr, const int32_t *__restrict__ b_col,
                          const int32_t *__restrict__ b_trans, int op_b, int nj, int inter4,
                          int64_t *__restrict__ cnt, const int64_t *__restrict__ off, int32_t *__restrict__ ea,
                          int32_t *__restrict__ eb, int32_t *__restrict__ rout, int segd, int32_t *__restrict__ seg)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nch) return;
    const int i = run_row[c];
    const int64_t p0 = run_p0[c];
    const int m = (int)min<int64_t>(nj, c_ptr[i + 1] - p0);
    int64_t pb[kMaxRun], eb_end[kMaxRun];
    for (int t = 0; t < m; ++t) {
        const int j = c_col[p0 + t];
        pb[t] = b_ptr[j];
        eb_end[t] = b_ptr[j + 1];
    }
    if (FILL)
        for (int t = 0; t < nj; ++t) rout[c * nj + t] = t < m ? (int32_t)(p0 + t) : -1;
    // With `seg` (runs of 2): the entries feeding both outputs first, then
    // those feeding only the first, then only the second (each in ascending
    // k); the count pass records the sizes of the first two segments.
    const int passes = segd ? 3 : 1;
    const int want[3] = {3, 1, 2};
    int64_t n = 0, o = FILL ? off[c] : 0;
    int64_t nseg[3] = {0, 0, 0};
    for (int pass = 0; pass < passes; ++pass) {
        for (int t = 0; t < m; ++t) pb[t] = b_ptr[c_col[p0 + t]];
        for (int64_t pa = a_ptr[i]; pa < a_ptr[i + 1]; ++pa) {
            const int k = a_col[pa];
            int mask = 0;
            for (int t = 0; t < m; ++t) {
                while (pb[t] < eb_end[t] && b_col[pb[t]] < k) ++pb[t];
                if (pb[t] < eb_end[t] && b_col[pb[t]] == k) mask |= 1 << t;
            }
            if (!mask || (segd && mask != want[pass])) continue;
            ++nseg[pass];
            if (FILL) {
                ea[o] = (int32_t)pa;
                for (int t = 0; t < nj; ++t) {
                    const int slot = inter4 ? (t & 3) * 4 + (t >> 2) : t;
                    int32_t v = -1;
                    // op(B)_kj: block (k, j) = trans of (j, k), or (j, k) itself for the conjugate transpose
                    if ((mask >> t) & 1) v = op_b ? (int32_t)pb[t] : b_trans[pb[t]];
                    eb[o * nj + slot] = v;
                }
                ++o;
            } else {
                ++n;
            }
        }
    }
    if (!FILL) {
        cnt[c] = n;
        if (seg) {
            seg[2 * c] = (int32_t)nseg[0];
            seg[2 * c + 1] = (int32_t)nseg[1];
        }
    }
}

void launch_run_count(hipStream_t s, int64_t nch, const int32_t *run_row, const int64_t *run_p0, const int64_t *c_ptr,
                      const int32_t *c_col, const int64_t *a_ptr, const int32_t *a_col, const int64_t *b_ptr,
                      const int32_t *b_col, int nj, int64_t *cnt, int32_t *seg)
{
    if (nch == 0) return;
    RT_CHECK(nj >= 1 && nj <= kMaxRun, RTDM_E_ARG, "row runs hold 1..16 outputs");
    RT_CHECK(!seg || nj == 2, RTDM_E_ARG, "segmented row runs hold 2 outputs");
    hipLaunchKernelGGL(k_run_sym<false>, dim3((unsigned)((nch + 127) / 128)), dim3(128), 0, s, nch, run_row, run_p0,
                       c_ptr, c_col, a_ptr, a_col, b_ptr, b_col, nullptr, 0, nj, 0, cnt, nullptr, nullptr, nullptr,
                       nullptr, seg ? 1 : 0, seg);
    RT_HIP(hipGetLastError());
}

void launch_run_fill(hipStream_t s, int64_t nch, const int32_t *run_row, const int64_t *run_p0, const int64_t *c_ptr,
                     const int32_t *c_col, const int64_t *a_ptr, const int32_t *a_col, const int64_t *b_ptr,
                     const int32_t *b_col, const int32_t *b_trans, int op_b, int nj, int inter4, const int64_t *off,
                     int32_t *ea, int32_t *eb, int32_t *rout, int segmented)
{
    if (nch == 0) return;
    RT_CHECK(nj >= 1 && nj <= kMaxRun, RTDM_E_ARG, "row runs hold 1..16 outputs");
    RT_CHECK(!segmented || (nj == 2 && !inter4), RTDM_E_ARG, "segmented row runs hold 2 outputs");
    hipLaunchKernelGGL(k_run_sym<true>, dim3((unsigned)((nch + 127) / 128)), dim3(128), 0, s, nch, run_row, run_p0,
                       c_ptr, c_col, a_ptr, a_col, b_ptr, b_col, b_trans, op_b, nj, inter4, nullptr, off, ea, eb,
                       rout, segmented ? 1 : 0, nullptr);
    RT_HIP(hipGetLastError());
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

// MFMA 16x16x4 f64 operand layout (wave of 64 lanes, lane = 16*q + r), as
// measured on gfx950:
//   A operand: lane supplies A[r][q]   (row r of the 16x4 slice, column q)
//   B operand: lane supplies B[q][r]   (row q of the 4x16 slice, column r)
//   D (4 doubles per lane): element e of lane is D[4*e + q][r]
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
        const int row = 4 * e + q, col = r;
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

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// block index.  xcd_block() with remap = 1 renumbers them so that XCD x runs
// the contiguous range [x*per, (x+1)*per) of logical blocks: neighbouring
// output blocks, which share operand blocks, then meet in the same L2.  The
// grid is launched with 8*per blocks; logical indices >= the real count exit.
//
// remap > 1 deals chunks of `remap` consecutive logical blocks to the XCDs
// round-robin instead (chunk m to XCD m % 8), so that the XCDs work on
// neighbouring chunks at the same time; the grid is then a multiple of
// 8*remap (xcd_grid with the same remap).
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block(int64_t nblocks, int remap = 1)
{
    if (!remap) return blockIdx.x;
    const int64_t x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
    if (remap > 1) return ((i / remap) * kXcds + x) * remap + i % remap;
    const int64_t per = (nblocks + kXcds - 1) / kXcds;
    return x * per + i;
}
static inline unsigned xcd_grid(int64_t nblocks, int remap = 1)
{
    const int64_t unit = remap > 1 ? (int64_t)kXcds * remap : kXcds;
    return (unsigned)(((nblocks + unit - 1) / unit) * unit);
}

// XCD mapping of the row-run kernels: the chunk size of the round-robin deal
// (128 workgroups: the XCDs then stream neighbouring outputs, whose operand
// blocks meet in the shared last-level cache; contiguous eighths measured
// 11 % slower at b = 13).
static int xcd_chunk() { return 128; }
// The same deal in chunks of about as many output blocks (1,024) for a kernel
// with `per_wg` output blocks per workgroup.
static int xcd_chunk_wg(int per_wg) { return std::max(2, xcd_chunk() * 8 / std::max(per_wg, 1)); }
// The b = 4 run kernels keep the hardware order (the deal changed their rate by
// under 2 % either way).
static int b4_chunk() { return 0; }

// Matrix-core step on one 16x16 tile: FP64 (v_mfma_f64_16x16x4_f64) or
// FP32 (v_mfma_f32_16x16x4_f32).  Both take A[r][q] / B[q][r] from lane
// 16*q + r; element e of the result sits in row 4*e + q for FP64 and in row
// 4*q + e for FP32 (measured on gfx950).
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <class T> struct Mfma16;
template <> struct Mfma16<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ inline acc_t step(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int e, int q) { return 4 * e + q; }
};
template <> struct Mfma16<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ inline acc_t step(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int e, int q) { return 4 * q + e; }
};

// TA / TB: the stored block is read transposed (op(A)[r][m] at m*B + r, op(B)[m][r]
// at r*B + m); CJA / CJB: conjugate; LC: write the output block column-major.
// A conjugate transpose of a row-major block is TA = CJA = 1; a column-major
// copy of a left operand is TA = 1, CJA = 0, so that the 16 lanes of a row
// group read contiguous doubles.
template <int B, bool AC, bool BC, int TA, int TB, class T = double, int CJA = TA, int CJB = TB,
          int LC = 0>
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
    const int oa_r = TA ? r : r * B;           // + m * (TA ? B : 1)
    const int ob_r = TB ? r * B : r;           // + m * (TB ? 1 : B)
    constexpr int sa = TA ? B : 1, sb = TB ? 1 : B;

    int tt = 0, m = q;                         // B >= 4: the first step stays in triple 0
    int2 ab = nt > 0 ? trip[t0] : make_int2(0, 0);
    T xar = 0, xai = 0, xbr = 0, xbi = 0;
    auto fetch = [&](T &far, T &fai, T &fbr, T &fbi) {
        far = fai = fbr = fbi = 0;
        if (tt < nt && rv) {
            const int64_t pa = (int64_t)ab.x * BB + oa_r + m * sa;
            const int64_t pb = (int64_t)ab.y * BB + ob_r + m * sb;
            far = (T)ar[pa];
            fbr = (T)br[pb];
            if (AC) fai = (T)(CJA ? -ai[pa] : ai[pa]);
            if (BC) fbi = (T)(CJB ? -bi[pb] : bi[pb]);
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
    typedef typename Mfma16<T>::acc_t acc_t;
    acc_t rr = {0, 0, 0, 0}, ii = {0, 0, 0, 0}, ri = {0, 0, 0, 0}, ir = {0, 0, 0, 0};
    fetch(xar, xai, xbr, xbi);
    for (int s = 0; s < steps; ++s) {
        advance();
        T nar, nai, nbr, nbi;
        fetch(nar, nai, nbr, nbi);
        rr = Mfma16<T>::step(xar, xbr, rr);
        if (AC && BC) ii = Mfma16<T>::step(xai, xbi, ii);
        if (BC) ri = Mfma16<T>::step(xar, xbi, ri);
        if (AC) ir = Mfma16<T>::step(xai, xbr, ir);
        xar = nar;
        xai = nai;
        xbr = nbr;
        xbi = nbi;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = Mfma16<T>::row(e, q), col = r;
        if (row < B && col < B) {
            const double re = (double)rr[e] - (double)ii[e];
            const double im = (double)ri[e] + (double)ir[e];
            const int64_t o = c * BB + (LC ? col * B + row : row * B + col);
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

// Step products, B = 13 or 16: the contraction of one output block runs over
// groups of four triples.  In each 4-wide MFMA step the lane group q (16
// lanes) supplies element s of the group's q-th triple, so B steps consume
// the four triples exactly (the order of the contraction sum is the only
// difference from a triple-by-triple loop).  The left operand is a
// column-major copy (op(A)[r][s] at s*B + r) and the right operand has
// op(B)[s][r] at s*B + r, so every load is a per-group base pointer plus a
// compile-time offset; lanes without data (rows r >= B, or past the last
// triple) point at a zero block.  Conjugation is a sign applied to the
// accumulated imaginary products at the end.
//
// T = float runs the same dataflow on the FP32 matrix cores (operands rounded
// to FP32 on load, FP32 accumulation).
template <int B, bool AC, bool BC, int CJA, int CJB, int LC, int WPB = 4, class T = double>
__global__ __launch_bounds__(64 * WPB) void k_spgemm_q4(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, double alr,
    double ali, const double *__restrict__ zero, const int32_t *__restrict__ order, int remap)
{
    static_assert(B >= 4 && B <= 16, "k_spgemm_q4 needs 4 <= B <= 16");
    constexpr int BB = B * B;
    const int lane = threadIdx.x & 63;
    const int64_t w = xcd_block((nout + WPB - 1) / WPB, remap) * WPB + (threadIdx.x >> 6);
    if (w >= nout) return;                     // uniform across the wave
    const int64_t c = order ? (int64_t)order[w] : w;
    const int r = lane & 15, q = lane >> 4;
    const bool rv = r < B;
    const int64_t t0 = off[c];
    const int nt = (int)(off[c + 1] - t0);
    typedef typename Mfma16<T>::acc_t acc_t;
    acc_t rr = {0, 0, 0, 0}, ii = {0, 0, 0, 0}, ri = {0, 0, 0, 0}, ir = {0, 0, 0, 0};
    for (int g = 0; g < nt; g += 4) {
        const double *pa = zero, *pai = zero, *pb = zero, *pbi = zero;
        if (rv && g + q < nt) {
            const int2 ab = trip[t0 + g + q];
            const int64_t oa = (int64_t)ab.x * BB + r, ob = (int64_t)ab.y * BB + r;
            pa = ar + oa;
            pb = br + ob;
            if (AC) pai = ai + oa;
            if (BC) pbi = bi + ob;
        }
#pragma unroll
        for (int st = 0; st < B; ++st) {
            const T xa = (T)pa[st * B], xb = (T)pb[st * B];
            rr = Mfma16<T>::step(xa, xb, rr);
            if (AC && BC) ii = Mfma16<T>::step((T)pai[st * B], (T)pbi[st * B], ii);
            if (BC) ri = Mfma16<T>::step(xa, (T)pbi[st * B], ri);
            if (AC) ir = Mfma16<T>::step((T)pai[st * B], xb, ir);
        }
    }
    // op(A)_im = sa * A_im, op(B)_im = sb * B_im
    constexpr double sa = CJA ? -1.0 : 1.0, sb = CJB ? -1.0 : 1.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = Mfma16<T>::row(e, q), col = r;
        if (row < B && col < B) {
            const double re = (double)rr[e] - (sa * sb) * (double)ii[e];
            const double im = sb * (double)ri[e] + sa * (double)ir[e];
            const int64_t o = c * BB + (LC ? col * B + row : row * B + col);
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

typedef __attribute__((address_space(1))) const double gdouble;

// Row runs of the step products: one wave computes NJ output blocks C_ij of
// the same row i.  The entries of the run are the contraction indices k used
// by any of its outputs; lane group q takes entry g + q, loads op(A)_ik once
// and op(B)_kj of every output (the zero block where that output has no
// triple with this k), and each loaded A element feeds NJ MFMAs.  The operand
// blocks of A beyond L2 are then fetched once per run instead of once per
// output; the price is the absent (zero) products of a run.  Data layout,
// lane mapping, conjugation and output as in k_spgemm_q4.
// seg (runs of 2, optional): per run the number of entries that feed both
// outputs (seg[2c]) and only the first (seg[2c+1]); the entries are stored in
// that order, the rest feed only the second.  Each segment then runs with
// only its outputs' products, so no matrix work goes to absent entries.
template <int B, bool AC, bool BC, int CJB, int LC, int NJ, class T = double, int MINW = 1>
__global__ __launch_bounds__(256, MINW) void k_spgemm_q4j(
    int64_t nch, const int64_t *__restrict__ off, const int32_t *__restrict__ ea,
    const int32_t *__restrict__ eb, const int32_t *__restrict__ cout,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, double alr,
    double ali, const double *__restrict__ zero, const int32_t *__restrict__ order, int remap,
    const int32_t *__restrict__ seg)
{
    static_assert(B >= 4 && B <= 16, "k_spgemm_q4j needs 4 <= B <= 16");
    constexpr int BB = B * B;
    const int lane = threadIdx.x & 63;
    const int64_t w = xcd_block((nch + 3) / 4, remap) * 4 + (threadIdx.x >> 6);
    if (w >= nch) return;                      // uniform across the wave
    const int64_t c = order ? (int64_t)order[w] : w;
    const int r = lane & 15, q = lane >> 4;
    const bool rv = r < B;
    const int64_t e0 = off[c];
    const int ne = (int)(off[c + 1] - e0);
    typedef typename Mfma16<T>::acc_t acc_t;
    acc_t rr[NJ], ri[NJ], ir[NJ];
#pragma unroll
    for (int t = 0; t < NJ; ++t) rr[t] = ri[t] = ir[t] = acc_t{0, 0, 0, 0};
    const gdouble *gz = (const gdouble *)zero;
    // entries [gb, ge) of the run; output t's products only where bit t of ACT is set
    auto groups = [&](int gb, int ge, auto act) {
        constexpr int ACT = decltype(act)::value;
        for (int g = gb; g < ge; g += 4) {
            // global-address-space pointers: the loads stay global loads (flat
            // loads would make every wait drain the scalar-memory counter too)
            const gdouble *pa = gz, *pai = gz;
            const gdouble *pb[NJ], *pbi[NJ];
#pragma unroll
            for (int t = 0; t < NJ; ++t) pb[t] = pbi[t] = gz;
            if (rv && g + q < ge) {
                const int64_t e = e0 + g + q;
                const int64_t oa = (int64_t)ea[e] * BB + r;
                pa = (const gdouble *)(ar + oa);
                if (AC) pai = (const gdouble *)(ai + oa);
#pragma unroll
                for (int t = 0; t < NJ; ++t) {
                    if (!((ACT >> t) & 1)) continue;
                    const int kb = eb[e * NJ + t];
                    if (kb >= 0) {
                        const int64_t ob = (int64_t)kb * BB + r;
                        pb[t] = (const gdouble *)(br + ob);
                        if (BC) pbi[t] = (const gdouble *)(bi + ob);
                    }
                }
            }
#pragma unroll
            for (int st = 0; st < B; ++st) {
                const T xa = (T)pa[st * B];
                const T xai = AC ? (T)pai[st * B] : (T)0;
                if constexpr (AC && BC) {
                    // two accumulators per output: re += a_r b_r + (-s a_i) b_i,
                    // im += (s a_r) b_i + a_i b_r with s = -1 for a conjugated B
                    const T nai = CJB ? xai : -xai, sar = CJB ? -xa : xa;
#pragma unroll
                    for (int t = 0; t < NJ; ++t) {
                        if (!((ACT >> t) & 1)) continue;
                        const T xb = (T)pb[t][st * B], xbi = (T)pbi[t][st * B];
                        rr[t] = Mfma16<T>::step(xa, xb, rr[t]);
                        ri[t] = Mfma16<T>::step(sar, xbi, ri[t]);
                        rr[t] = Mfma16<T>::step(nai, xbi, rr[t]);
                        ri[t] = Mfma16<T>::step(xai, xb, ri[t]);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < NJ; ++t) {
                        if (!((ACT >> t) & 1)) continue;
                        const T xb = (T)pb[t][st * B];
                        const T xbi = BC ? (T)pbi[t][st * B] : (T)0;
                        rr[t] = Mfma16<T>::step(xa, xb, rr[t]);
                        if (BC) ri[t] = Mfma16<T>::step(xa, xbi, ri[t]);
                        if (AC) ir[t] = Mfma16<T>::step(xai, xb, ir[t]);
                    }
                }
            }
        }
    };
    constexpr int ALL = (1 << NJ) - 1;
    if constexpr (NJ == 2) {
        if (seg) {
            const int nf = seg[2 * c], n0 = seg[2 * c + 1];   // uniform across the wave
            groups(0, nf, std::integral_constant<int, 3>());
            groups(nf, nf + n0, std::integral_constant<int, 1>());
            groups(nf + n0, ne, std::integral_constant<int, 2>());
        } else {
            groups(0, ne, std::integral_constant<int, ALL>());
        }
    } else {
        groups(0, ne, std::integral_constant<int, ALL>());
    }
    constexpr double sb = CJB ? -1.0 : 1.0;
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
        const int p = cout[c * NJ + t];
        if (p < 0) continue;                   // uniform: a short run
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = Mfma16<T>::row(e, q), col = r;
            if (row < B && col < B) {
                const double re = (double)rr[t][e];
                const double im = (AC && BC) ? (double)ri[t][e] : sb * (double)ri[t][e] + (double)ir[t][e];
                const int64_t o = (int64_t)p * BB + (LC ? col * B + row : row * B + col);
                cr[o] = alr * re - ali * im;
                if (ci) ci[o] = alr * im + ali * re;
            }
        }
    }
}

// b = 4: v_mfma_f64_4x4x4_4b_f64 runs four independent 4x4x4 products, one
// per "MFMA block".  Each output block needs SUB real sub-products (1: real x
// real; 2: one operand complex; 4: complex x complex: re*re, im*im, re*im,
// im*re), so a wave serves 4/SUB output blocks, each on SUB MFMA blocks, with
// no padding anywhere: one instruction per step does one block triple of 4/SUB
// outputs.  Lane layout (measured on gfx950), lane = 16*q + 4*g + r:
//   MFMA block g; A operand A_g[r][q]; B operand B_g[q][r]; D: D_g[q][r].
// The wave's outputs advance in lock-step over their triple lists; a finished
// output feeds zeros.

// Split-precision block products (B = 4 or 13, operand layouts as in
// k_spgemm_kc).  Each FP64 operand element x is split into two 16-bit
// parts and the product of two elements is taken as three 16-bit products
// with FP32 accumulation on the matrix cores (v_mfma_f32_16x16x32_*):
//   MODE 0, BF16 x3 (the three-product split of Henry, Tang and Heinecke,
//     2019): hi = bf16(x), lo = bf16(x - hi); a b ~ ah bh + ah bl + al bh.
//   MODE 1, FP16 x2 (the scaled split of Ootomo and Yokota, 2022):
//     y = x s with s = 2^(13 - floor(log2 max|X|)) per operand matrix,
//     hi = fp16(y), lo = fp16((y - hi) 2^11);
//     a b ~ (ah bh + (ah bl + al bh) 2^-11) / (sa sb).
// The contraction of an output block is concatenated over its triples; a
// 32-wide MFMA step takes elements 8q..8q+7 of the step from lane group q.
// The sign of a conjugated operand's imaginary part is applied at the load.
template <int MODE> struct Split16;
template <> struct Split16<0> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    static __device__ inline void split(double x, float, __bf16 &hi, __bf16 &lo)
    {
        float xf = (float)x;
        asm volatile("" : "+v"(xf));
        hi = (__bf16)xf;
        lo = (__bf16)(xf - (float)hi);
    }
    static __device__ inline f32x4 mfma(v8 a, v8 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    typedef __bf16 e_t;
};
template <> struct Split16<1> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    static __device__ inline void split(double x, float sc, _Float16 &hi, _Float16 &lo)
    {
        const float y = (float)x * sc;
        hi = (_Float16)y;
        lo = (_Float16)((y - (float)hi) * 2048.0f);
    }
    static __device__ inline f32x4 mfma(v8 a, v8 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    typedef _Float16 e_t;
};

// Power-of-two operand scale of the FP16 split from max |X| (both planes).
__device__ inline float f16_scale(const double *mx, int k)
{
    const double m = fmax(mx[8 * k + 3], mx[8 * k + 7]);
    return m > 0.0 ? ldexpf(1.0f, 13 - ilogb(m)) : 1.0f;
}

template <int B, bool AC, bool BC, int TA, int TB, int MODE>
__global__ __launch_bounds__(256) void k_spgemm_split(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, double alr,
    double ali, const double *__restrict__ maxabs)
{
    typedef Split16<MODE> SP;
    typedef typename SP::v8 v8;
    constexpr int BB = B * B;
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nout) return;                     // uniform across the wave
    const int r = lane & 15, q = lane >> 4;
    const bool rv = r < B;
    const int64_t t0 = off[c];
    const int nt = (int)(off[c + 1] - t0);
    const int L = nt * B;
    const float sa = MODE ? f16_scale(maxabs, 0) : 1.0f;
    const float sb = MODE ? f16_scale(maxabs, 1) : 1.0f;
    f32x4 h[4] = {}, m[4] = {};                // rr, ii, ri, ir: hi*hi and the mixed terms
    for (int u0 = 0; u0 < L; u0 += 32) {
        v8 ahr, alr8, ahi, ali8, bhr, blr8, bhi, bli8;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int u = u0 + 8 * q + v;
            double xar = 0.0, xai = 0.0, xbr = 0.0, xbi = 0.0;
            if (rv && u < L) {
                const int tt = u / B, k = u - tt * B;
                const int2 ab = trip[t0 + tt];
                const int64_t pa = (int64_t)ab.x * BB + (TA ? k * B + r : r * B + k);
                const int64_t pb = (int64_t)ab.y * BB + (TB ? r * B + k : k * B + r);
                xar = ar[pa];
                xbr = br[pb];
                if (AC) xai = TA ? -ai[pa] : ai[pa];
                if (BC) xbi = TB ? -bi[pb] : bi[pb];
            }
            typename SP::e_t hi, lo;
            SP::split(xar, sa, hi, lo); ahr[v] = hi; alr8[v] = lo;
            SP::split(xbr, sb, hi, lo); bhr[v] = hi; blr8[v] = lo;
            if (AC) { SP::split(xai, sa, hi, lo); ahi[v] = hi; ali8[v] = lo; }
            if (BC) { SP::split(xbi, sb, hi, lo); bhi[v] = hi; bli8[v] = lo; }
        }
        auto prod3 = [&](int k, const v8 &ah, const v8 &al, const v8 &bh, const v8 &bl) {
            h[k] = SP::mfma(ah, bh, h[k]);
            m[k] = SP::mfma(ah, bl, m[k]);
            m[k] = SP::mfma(al, bh, m[k]);
        };
        prod3(0, ahr, alr8, bhr, blr8);
        if (AC && BC) prod3(1, ahi, ali8, bhi, bli8);
        if (BC) prod3(2, ahr, alr8, bhi, bli8);
        if (AC) prod3(3, ahi, ali8, bhr, blr8);
    }
    const double inv = 1.0 / ((double)sa * (double)sb);
    const double ml = MODE ? 1.0 / 2048.0 : 1.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = 4 * q + e, col = r;
        if (row < B && col < B) {
            double v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = ((double)h[k][e] + ml * (double)m[k][e]) * inv;
            const double re = v[0] - v[1];
            const double im = v[2] + v[3];
            const int64_t o = c * BB + row * B + col;
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

// Split-precision variant of k_spgemm_q4 for real operands (the Taylor-term
// products A tau of the *_TAYLOR forms), same four-triple grouping, order and
// XCD mapping.  Each 16-bit MFMA (v_mfma_f32_16x16x16_{bf16,f16}) step takes
// four consecutive contraction elements s0..s0+3 of its triple from lane
// group q, so four steps cover B = 13 (elements 13..15 are zero).  Every
// FP64 element is split as in k_spgemm_split (BF16 hi/lo, or FP16 hi/lo of
// the power-of-two scaled value with the low part scaled by 2^11) and each
// product is taken as hi*hi + hi*lo + lo*hi with FP32 accumulation.
template <int MODE> struct Split4;
template <> struct Split4<0> {
    typedef short v4 __attribute__((ext_vector_type(4)));
    static __device__ inline void split(double x, float, short &hi, short &lo)
    {
        float xf = (float)x;                       // 24 bits hold both 8-bit parts
        asm volatile("" : "+v"(xf));               // round to FP32 first: keeps the conversions apart
        const __bf16 h = (__bf16)xf;
        const __bf16 l = (__bf16)(xf - (float)h);
        hi = __builtin_bit_cast(short, h);
        lo = __builtin_bit_cast(short, l);
    }
    static __device__ inline f32x4 mfma(v4 a, v4 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    typedef short e_t;
};
template <> struct Split4<1> {
    typedef _Float16 v4 __attribute__((ext_vector_type(4)));
    static __device__ inline void split(double x, float sc, _Float16 &hi, _Float16 &lo)
    {
        const float y = (float)x * sc;              // sc a power of two; 24 bits hold both 11-bit parts
        hi = (_Float16)y;
        lo = (_Float16)((y - (float)hi) * 2048.0f);
    }
    static __device__ inline f32x4 mfma(v4 a, v4 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
    typedef _Float16 e_t;
};

template <int B, int MODE, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_spgemm_q4s(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip, const double *__restrict__ ar,
    const double *__restrict__ br, double *__restrict__ cr, double alr, const double *__restrict__ zero,
    const int32_t *__restrict__ order, const double *__restrict__ maxabs, int remap)
{
    typedef Split4<MODE> SP;
    typedef typename SP::v4 v4;
    constexpr int BB = B * B;
    const int lane = threadIdx.x & 63;
    const int64_t w = xcd_block((nout + WPB - 1) / WPB, remap) * WPB + (threadIdx.x >> 6);
    if (w >= nout) return;                     // uniform across the wave
    const int64_t c = order ? (int64_t)order[w] : w;
    const int r = lane & 15, q = lane >> 4;
    const bool rv = r < B;
    const int64_t t0 = off[c];
    const int nt = (int)(off[c + 1] - t0);
    const float sa = MODE ? f16_scale(maxabs, 0) : 1.0f;
    const float sb = MODE ? f16_scale(maxabs, 1) : 1.0f;
    f32x4 h = {0, 0, 0, 0}, m = {0, 0, 0, 0};
    for (int g = 0; g < nt; g += 4) {
        const double *pa = zero, *pb = zero;
        if (rv && g + q < nt) {
            const int2 ab = trip[t0 + g + q];
            pa = ar + (int64_t)ab.x * BB + r;
            pb = br + (int64_t)ab.y * BB + r;
        }
#pragma unroll
        for (int s0 = 0; s0 < B; s0 += 4) {
            v4 ah, al, bh, bl;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int st = s0 + v;
                const double xa = st < B ? pa[st * B] : 0.0, xb = st < B ? pb[st * B] : 0.0;
                typename SP::e_t hi, lo;
                SP::split(xa, sa, hi, lo);
                ah[v] = hi;
                al[v] = lo;
                SP::split(xb, sb, hi, lo);
                bh[v] = hi;
                bl[v] = lo;
            }
            h = SP::mfma(ah, bh, h);
            m = SP::mfma(ah, bl, m);
            m = SP::mfma(al, bh, m);
        }
    }
    const double inv = 1.0 / ((double)sa * (double)sb);
    const double ml = MODE ? 1.0 / 2048.0 : 1.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = 4 * q + e, col = r;
        if (row < B && col < B) cr[c * BB + row * B + col] = alr * (((double)h[e] + ml * (double)m[e]) * inv);
    }
}

void launch_spgemm_cm_split(hipStream_t s, const SpgemmArgs &a)
{
    if (a.nout == 0) return;
    RT_CHECK(a.b == 13 && !a.ai && !a.bi && !a.ci &&
                 (a.precision == RTDM_PREC_BF16X3 || a.precision == RTDM_PREC_FP16X2),
             RTDM_E_UNSUPPORTED, "split step products need b = 13, real operands and a split precision");
    RT_CHECK(a.precision != RTDM_PREC_FP16X2 || a.maxabs, RTDM_E_ARG, "FP16 split products need operand maxima");
    const int wpb = a.wpb;
    const int remap = xcd_chunk_wg(wpb);
    const unsigned grid = xcd_grid((a.nout + wpb - 1) / wpb, remap);
#define RT_Q4S(M, W)                                                                                      \
    hipLaunchKernelGGL((k_spgemm_q4s<13, M, W>), dim3(grid), dim3(64 * W), 0, s, a.nout, a.off, a.trip, a.ar, \
                       a.br, a.cr, a.alpha_re, a.zero, a.order, a.maxabs, remap)
    const int mode = a.precision == RTDM_PREC_FP16X2 ? 1 : 0;
    if (mode == 0) {
        if (wpb == 16) RT_Q4S(0, 16);
        else if (wpb == 8) RT_Q4S(0, 8);
        else RT_Q4S(0, 4);
    } else {
        if (wpb == 16) RT_Q4S(1, 16);
        else if (wpb == 8) RT_Q4S(1, 8);
        else RT_Q4S(1, 4);
    }
#undef RT_Q4S
    RT_HIP(hipGetLastError());
}

template <int SUB, bool AC, bool BC, int OPA, int OPB>
__global__ __launch_bounds__(256) void k_spgemm_b4(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, double alr,
    double ali)
{
    constexpr int OUT = 4 / SUB;               // outputs per wave
    const int lane = threadIdx.x & 63;
    const int g = (lane >> 2) & 3, r = lane & 3, q = lane >> 4;
    const int sub = g % SUB;                   // which real sub-product this MFMA block runs
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t c0 = wave * OUT;
    if (c0 >= nout) return;                    // uniform across the wave
    const int64_t c = c0 + g / SUB;            // this lane's output block
    const bool live = c < nout;
    const int64_t t0 = live ? off[c] : 0;
    const int nt = live ? (int)(off[c + 1] - t0) : 0;
    // longest list of the wave (the four MFMA blocks sit 4 lanes apart)
    int ntmax = max(nt, __shfl_xor(nt, 4, 64));
    ntmax = max(ntmax, __shfl_xor(ntmax, 8, 64));
    // operand planes of this sub-product: sub 0 re*re, 1 im*im, 2 re*im, 3 im*re (SUB = 4);
    // SUB = 2: sub 0 re*re, sub 1 the product with the complex operand's imaginary part.
    bool a_im = false, b_im = false;
    if (SUB == 4) { a_im = (sub == 1 || sub == 3); b_im = (sub == 1 || sub == 2); }
    if (SUB == 2) { a_im = AC && sub == 1; b_im = BC && sub == 1; }
    const double *pa = a_im ? ai : ar;
    const double *pb = b_im ? bi : br;
    const double sa = (a_im && OPA) ? -1.0 : 1.0;
    const double sb = (b_im && OPB) ? -1.0 : 1.0;
    const int ia = OPA ? (q * 4 + r) : (r * 4 + q);   // op(A)[r][q]
    const int ib = OPB ? (r * 4 + q) : (q * 4 + r);   // op(B)[q][r]
    double acc = 0.0;
    double xa = 0.0, xb = 0.0;
    if (nt > 0) {
        const int2 ab = trip[t0];
        xa = sa * pa[(int64_t)ab.x * 16 + ia];
        xb = sb * pb[(int64_t)ab.y * 16 + ib];
    }
    for (int t = 0; t < ntmax; ++t) {
        double na = 0.0, nb = 0.0;
        if (t + 1 < nt) {
            const int2 ab = trip[t0 + t + 1];
            na = sa * pa[(int64_t)ab.x * 16 + ia];
            nb = sb * pb[(int64_t)ab.y * 16 + ib];
        }
        acc = __builtin_amdgcn_mfma_f64_4x4x4f64(xa, xb, acc, 0, 0, 0);
        xa = na;
        xb = nb;
    }
    // combine the sub-products of each output (MFMA blocks are 4 lanes apart)
    double re = acc, im = 0.0;
    if (SUB == 4) {
        const double d1 = __shfl_down(acc, 4, 64);    // block g+1
        const double d2 = __shfl_down(acc, 8, 64);    // block g+2
        const double d3 = __shfl_down(acc, 12, 64);   // block g+3
        re = acc - d1;
        im = d2 + d3;
    } else if (SUB == 2) {
        im = __shfl_down(acc, 4, 64);
    }
    if (live && sub == 0) {
        const int64_t o = c * 16 + q * 4 + r;
        cr[o] = alr * re - ali * im;
        if (ci) ci[o] = alr * im + ali * re;
    }
}




// Reduced-precision products for b = 4 on the 16-block 4x4 matrix-core
// instructions (gfx950, measured layout: lane 4 blk + r supplies row r of
// A_blk and column r of B_blk, and holds D_blk[e][r] in its value e).  A wave
// runs 16 output blocks, one per MFMA block, one triple of each per step:
//   MODE 0 FP32   : four v_mfma_f32_4x4x1_16b per block product;
//   MODE 1 BF16x3 : hi/lo split, three v_mfma_f32_4x4x4_16b_bf16;
//   MODE 2 FP16x2 : scaled hi/lo split, three v_mfma_f32_4x4x4_16b_f16.
// Operands are FP64 in memory (op(A) = A; op(B) = B or B^dagger), results
// FP64; accumulation FP32.
template <int MODE> struct Small4;
template <> struct Small4<1> {
    typedef short v4 __attribute__((ext_vector_type(4)));
    static __device__ inline f32x4 mfma(v4 a, v4 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
    }
    static __device__ inline void split(double x, float, short &hi, short &lo) { Split4<0>::split(x, 1.0f, hi, lo); }
    typedef short e_t;
};
template <> struct Small4<2> {
    typedef _Float16 v4 __attribute__((ext_vector_type(4)));
    static __device__ inline f32x4 mfma(v4 a, v4 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_4x4x4f16(a, b, c, 0, 0, 0);
    }
    static __device__ inline void split(double x, float sc, _Float16 &hi, _Float16 &lo)
    {
        Split4<1>::split(x, sc, hi, lo);
    }
    typedef _Float16 e_t;
};

//
// RUNS: the wave computes a row run of 16 outputs (SpgemmArgs::ch_*, b = 4
// slot order) instead of 16 consecutive outputs: all blocks share the entry's
// op(A)_ik, and block blk takes the op(B)_kj of output blk (zero if absent).
template <bool AC, bool BC, int OPB, int MODE, bool RUNS = false>
__global__ __launch_bounds__(256) void k_spgemm_b4x(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, double alr, double ali,
    const double *__restrict__ maxabs, const int32_t *__restrict__ ea = nullptr,
    const int32_t *__restrict__ eb = nullptr, const int32_t *__restrict__ rout = nullptr)
{
    const int lane = threadIdx.x & 63;
    const int blk = lane >> 2, r = lane & 3;
    // RUNS: nout is the number of runs, off the entry offsets
    const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t c0 = RUNS ? wv : wv * 16;
    if (c0 >= nout) return;                    // uniform across the wave
    const int64_t c = RUNS ? (int64_t)rout[wv * 16 + blk] : c0 + blk;
    const bool live = RUNS ? c >= 0 : c < nout;
    const int64_t t0 = RUNS ? off[wv] : (live ? off[c] : 0);
    const int nt = RUNS ? (int)(off[wv + 1] - t0) : (live ? (int)(off[c + 1] - t0) : 0);
    int ntmax = nt;
    if (!RUNS) {
#pragma unroll
        for (int o = 4; o < 64; o <<= 1) ntmax = max(ntmax, __shfl_xor(ntmax, o, 64));
    }
    const int slot = (blk & 3) * 4 + (blk >> 2);
    const float sa = MODE == 2 ? f16_scale(maxabs, 0) : 1.0f;
    const float sb = MODE == 2 ? f16_scale(maxabs, 1) : 1.0f;
    f32x4 h[4] = {}, m[4] = {};                // rr, ii, ri, ir
    const double cb = OPB ? -1.0 : 1.0;
    for (int t = 0; t < ntmax; ++t) {
        double xa[4] = {0, 0, 0, 0}, xai[4] = {0, 0, 0, 0}, xb[4] = {0, 0, 0, 0}, xbi[4] = {0, 0, 0, 0};
        int2 ab = make_int2(0, -1);
        if (RUNS) ab = make_int2(ea[t0 + t], eb[(t0 + t) * 16 + slot]);
        else if (t < nt) ab = trip[t0 + t];
        if (ab.y >= 0) {
            const int64_t pa = (int64_t)ab.x * 16 + r * 4, pb = (int64_t)ab.y * 16;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                xa[k] = ar[pa + k];                                    // A[r][k]
                const int64_t e = OPB ? pb + r * 4 + k : pb + k * 4 + r; // op(B)[k][r]
                xb[k] = br[e];
                if (AC) xai[k] = ai[pa + k];
                if (BC) xbi[k] = cb * bi[e];
            }
        }
        if (MODE == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                h[0] = __builtin_amdgcn_mfma_f32_4x4x1f32((float)xa[k], (float)xb[k], h[0], 0, 0, 0);
                if (AC && BC) h[1] = __builtin_amdgcn_mfma_f32_4x4x1f32((float)xai[k], (float)xbi[k], h[1], 0, 0, 0);
                if (BC) h[2] = __builtin_amdgcn_mfma_f32_4x4x1f32((float)xa[k], (float)xbi[k], h[2], 0, 0, 0);
                if (AC) h[3] = __builtin_amdgcn_mfma_f32_4x4x1f32((float)xai[k], (float)xb[k], h[3], 0, 0, 0);
            }
        } else {
            typedef Small4<MODE == 0 ? 1 : MODE> SP;
            typedef typename SP::v4 v4;
            auto prod3 = [&](int u, const double *x, float sx, const double *y, float sy) {
                v4 xh, xl, yh, yl;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    typename SP::e_t hi, lo;
                    SP::split(x[k], sx, hi, lo);
                    xh[k] = hi;
                    xl[k] = lo;
                    SP::split(y[k], sy, hi, lo);
                    yh[k] = hi;
                    yl[k] = lo;
                }
                h[u] = SP::mfma(xh, yh, h[u]);
                m[u] = SP::mfma(xh, yl, m[u]);
                m[u] = SP::mfma(xl, yh, m[u]);
            };
            prod3(0, xa, sa, xb, sb);
            if (AC && BC) prod3(1, xai, sa, xbi, sb);
            if (BC) prod3(2, xa, sa, xbi, sb);
            if (AC) prod3(3, xai, sa, xb, sb);
        }
    }
    if (!live) return;
    const double inv = 1.0 / ((double)sa * (double)sb);
    const double ml = MODE == 2 ? 1.0 / 2048.0 : (MODE == 1 ? 1.0 : 0.0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = ((double)h[u][e] + ml * (double)m[u][e]) * inv;
        const double re = v[0] - v[1], im = v[2] + v[3];
        const int64_t o = c * 16 + e * 4 + r;
        cr[o] = alr * re - ali * im;
        if (ci) ci[o] = alr * im + ali * re;
    }
}

template <bool AC, bool BC, int OB>
static void launch_b4x(hipStream_t s, const SpgemmArgs &a)
{
    if (a.nch > 0) {
        RT_CHECK(a.nj == 16, RTDM_E_ARG, "b = 4 row runs hold 16 outputs");
        const dim3 g((unsigned)((a.nch + 3) / 4)), t(256);
#define RT_B4XJ(M)                                                                                      \
    hipLaunchKernelGGL((k_spgemm_b4x<AC, BC, OB, M, true>), g, t, 0, s, a.nch, a.ch_off, a.trip, a.ar, a.ai, \
                       a.br, a.bi, a.cr, a.ci, a.alpha_re, a.alpha_im, a.maxabs, a.ch_a, a.ch_b, a.ch_out)
        if (a.precision == RTDM_PREC_FP32) RT_B4XJ(0);
        else if (a.precision == RTDM_PREC_BF16X3) RT_B4XJ(1);
        else RT_B4XJ(2);
#undef RT_B4XJ
        return;
    }
    const dim3 g((unsigned)((a.nout + 63) / 64)), t(256);
#define RT_B4X(M)                                                                                     \
    hipLaunchKernelGGL((k_spgemm_b4x<AC, BC, OB, M>), g, t, 0, s, a.nout, a.off, a.trip, a.ar, a.ai, a.br, \
                       a.bi, a.cr, a.ci, a.alpha_re, a.alpha_im, a.maxabs)
    if (a.precision == RTDM_PREC_FP32) RT_B4X(0);
    else if (a.precision == RTDM_PREC_BF16X3) RT_B4X(1);
    else RT_B4X(2);
#undef RT_B4X
}


// FP64 b = 4 product, 16 output blocks per wave: four v_mfma_f64_4x4x4_4b per
// triple step (instruction j runs outputs c0 + 4j + g in its four blocks), so
// every lane has eight (real) operand loads in flight per step instead of
// two.  Same operand bytes per triple as k_spgemm_b4.
template <bool AC, bool BC, int OPB>
__global__ __launch_bounds__(256) void k_spgemm_b4w(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const double *__restrict__ ar, const double *__restrict__ ai, const double *__restrict__ br,
    const double *__restrict__ bi, double *__restrict__ cr, double *__restrict__ ci, double alr, double ali)
{
    const int lane = threadIdx.x & 63;
    const int g = (lane >> 2) & 3, r = lane & 3, q = lane >> 4;
    const int64_t c0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (c0 >= nout) return;                    // uniform across the wave
    const int ia = r * 4 + q;                          // A[r][q]
    const int ib = OPB ? (r * 4 + q) : (q * 4 + r);    // op(B)[q][r]
    const double cb = OPB ? -1.0 : 1.0;
    int64_t t0[4];
    int nt[4];
    int ntmax = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t c = c0 + 4 * j + g;
        t0[j] = c < nout ? off[c] : 0;
        nt[j] = c < nout ? (int)(off[c + 1] - t0[j]) : 0;
        ntmax = max(ntmax, nt[j]);
    }
    ntmax = max(ntmax, __shfl_xor(ntmax, 4, 64));
    ntmax = max(ntmax, __shfl_xor(ntmax, 8, 64));
    double rr[4] = {0, 0, 0, 0}, ii[4] = {0, 0, 0, 0}, ri[4] = {0, 0, 0, 0}, ir[4] = {0, 0, 0, 0};
    for (int t = 0; t < ntmax; ++t) {
        double xar[4], xai[4], xbr[4], xbi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            xar[j] = xai[j] = xbr[j] = xbi[j] = 0.0;
            if (t < nt[j]) {
                const int2 ab = trip[t0[j] + t];
                const int64_t pa = (int64_t)ab.x * 16 + ia, pb = (int64_t)ab.y * 16 + ib;
                xar[j] = ar[pa];
                xbr[j] = br[pb];
                if (AC) xai[j] = ai[pa];
                if (BC) xbi[j] = cb * bi[pb];
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            rr[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xar[j], xbr[j], rr[j], 0, 0, 0);
            if (AC && BC) ii[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xai[j], xbi[j], ii[j], 0, 0, 0);
            if (BC) ri[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xar[j], xbi[j], ri[j], 0, 0, 0);
            if (AC) ir[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xai[j], xbr[j], ir[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t c = c0 + 4 * j + g;
        if (c < nout) {
            const double re = rr[j] - ii[j], im = ri[j] + ir[j];
            const int64_t o = c * 16 + q * 4 + r;
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

// The entries [e0, e1) (every `stride`-th) of one b = 4 row run, software
// pipelined (complex x complex only in the split form for few runs, where
// latency and not occupancy decides): the indices of entry e + 2 and the operands of
// entry e + 1 are requested before the products of entry e, so that a wave
// has the next entry's loads in flight while its products run (the loads
// return in order, so waiting for an entry's operands never waits for later
// requests).  The products are issued in the same order as a plain loop over
// the entries.
template <bool AC, bool BC, bool PIPE_CPLX>
__device__ inline void b4_run_entries(int64_t e0, int64_t e1, int stride, const int32_t *__restrict__ ea,
                                      const int32_t *__restrict__ eb, const double *__restrict__ ar,
                                      const double *__restrict__ ai, const double *__restrict__ br,
                                      const double *__restrict__ bi, int ia, int ib, int g, double cb,
                                      double rr[4], double ii[4], double ri[4], double ir[4])
{
    struct Ops {
        double xar, xai, xbr[4], xbi[4];
    };
    auto load_idx = [&](int64_t e, int &a, int4 &kb) {
        a = ea[e];
        kb = *reinterpret_cast<const int4 *>(eb + e * 16 + g * 4);
    };
    auto load_ops = [&](int a, int4 kb4, Ops &o) {
        const int64_t pa = (int64_t)a * 16 + ia;
        o.xar = ar[pa];
        o.xai = AC ? ai[pa] : 0.0;
        const int kb[4] = {kb4.x, kb4.y, kb4.z, kb4.w};
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            o.xbr[jj] = o.xbi[jj] = 0.0;
            if (kb[jj] >= 0) {
                const int64_t pb = (int64_t)kb[jj] * 16 + ib;
                o.xbr[jj] = br[pb];
                if (BC) o.xbi[jj] = cb * bi[pb];
            }
        }
    };
    if (e0 >= e1) return;
    if constexpr (AC && BC && !PIPE_CPLX) {
        // complex x complex over many runs: twice the operand registers; the
        // pipeline's extra set cost waves per SIMD and made these products
        // slower, so they take the entries one at a time
        for (int64_t e = e0; e < e1; e += stride) {
            int a;
            int4 kb;
            Ops o;
            load_idx(e, a, kb);
            load_ops(a, kb, o);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                rr[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(o.xar, o.xbr[jj], rr[jj], 0, 0, 0);
                ii[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(o.xai, o.xbi[jj], ii[jj], 0, 0, 0);
                ri[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(o.xar, o.xbi[jj], ri[jj], 0, 0, 0);
                ir[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(o.xai, o.xbr[jj], ir[jj], 0, 0, 0);
            }
        }
        return;
    }
    Ops cur, nxt;
    int a_n = 0;
    int4 kb_n = make_int4(-1, -1, -1, -1);
    {
        int a0;
        int4 k0;
        load_idx(e0, a0, k0);
        if (e0 + stride < e1) load_idx(e0 + stride, a_n, kb_n);
        load_ops(a0, k0, cur);
    }
    for (int64_t e = e0; e < e1; e += stride) {
        int a_nn = 0;
        int4 kb_nn = make_int4(-1, -1, -1, -1);
        if (e + 2 * stride < e1) load_idx(e + 2 * stride, a_nn, kb_nn);
        if (e + stride < e1) load_ops(a_n, kb_n, nxt);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            rr[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(cur.xar, cur.xbr[jj], rr[jj], 0, 0, 0);
            if (AC && BC) ii[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(cur.xai, cur.xbi[jj], ii[jj], 0, 0, 0);
            if (BC) ri[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(cur.xar, cur.xbi[jj], ri[jj], 0, 0, 0);
            if (AC) ir[jj] = __builtin_amdgcn_mfma_f64_4x4x4f64(cur.xai, cur.xbr[jj], ir[jj], 0, 0, 0);
        }
        cur = nxt;
        a_n = a_nn;
        kb_n = kb_nn;
    }
}

// FP64 b = 4 product over row runs of 16 outputs (SpgemmArgs::ch_*, slots in
// the lane order below): one wave per run.  Each entry k of the run is one
// triple step: every lane loads the same op(A)_ik element position (one
// block for the whole wave) and the op(B)_kj elements of its four outputs
// (zero where an output has no triple with this k); instruction jj of the
// four v_mfma_f64_4x4x4_4b runs outputs 4 jj + g in its blocks g.  Against
// k_spgemm_b4w the left-operand loads fall from one block per output and
// triple to one per entry; the price is the absent (zero) products.
template <bool AC, bool BC, int OPB>
__global__ __launch_bounds__(256) void k_spgemm_b4j(
    int64_t nch, const int64_t *__restrict__ off, const int32_t *__restrict__ ea,
    const int32_t *__restrict__ eb, const int32_t *__restrict__ cout, const double *__restrict__ ar,
    const double *__restrict__ ai, const double *__restrict__ br, const double *__restrict__ bi,
    double *__restrict__ cr, double *__restrict__ ci, double alr, double ali, int remap)
{
    const int lane = threadIdx.x & 63;
    const int g = (lane >> 2) & 3, r = lane & 3, q = lane >> 4;
    const int64_t c = xcd_block((nch + 3) / 4, remap) * 4 + (threadIdx.x >> 6);
    if (c >= nch) return;                      // uniform across the wave
    const int ia = r * 4 + q;                          // A[r][q]
    const int ib = OPB ? (r * 4 + q) : (q * 4 + r);    // op(B)[q][r]
    const double cb = OPB ? -1.0 : 1.0;
    double rr[4] = {0, 0, 0, 0}, ii[4] = {0, 0, 0, 0}, ri[4] = {0, 0, 0, 0}, ir[4] = {0, 0, 0, 0};
    b4_run_entries<AC, BC, false>(off[c], off[c + 1], 1, ea, eb, ar, ai, br, bi, ia, ib, g, cb, rr, ii, ri, ir);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int p = cout[c * 16 + 4 * jj + g];
        if (p >= 0) {
            const double re = rr[jj] - ii[jj], im = ri[jj] + ir[jj];
            const int64_t o = (int64_t)p * 16 + q * 4 + r;
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

// The same product for products with few runs (small systems): one
// workgroup of W waves per run, wave w taking the entries w, w + W, ..., so
// that a run's chain of dependent loads is 1/W as long and W times as many
// waves share the chip.  The waves' partial sums are added in LDS in the
// fixed order w = 0, 1, ..., W - 1.
template <bool AC, bool BC, int OPB, int W>
__global__ __launch_bounds__(64 * W) void k_spgemm_b4js(
    int64_t nch, const int64_t *__restrict__ off, const int32_t *__restrict__ ea,
    const int32_t *__restrict__ eb, const int32_t *__restrict__ cout, const double *__restrict__ ar,
    const double *__restrict__ ai, const double *__restrict__ br, const double *__restrict__ bi,
    double *__restrict__ cr, double *__restrict__ ci, double alr, double ali)
{
    constexpr int NACC = 1 + (AC && BC) + BC + AC;   // accumulators per output: rr, ii, ri, ir
    __shared__ double part[W - 1][NACC * 4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = (lane >> 2) & 3, r = lane & 3, q = lane >> 4;
    const int64_t c = blockIdx.x;              // grid = nch: uniform across the workgroup
    const int ia = r * 4 + q;
    const int ib = OPB ? (r * 4 + q) : (q * 4 + r);
    const double cb = OPB ? -1.0 : 1.0;
    double rr[4] = {0, 0, 0, 0}, ii[4] = {0, 0, 0, 0}, ri[4] = {0, 0, 0, 0}, ir[4] = {0, 0, 0, 0};
    b4_run_entries<AC, BC, true>(off[c] + wv, off[c + 1], W, ea, eb, ar, ai, br, bi, ia, ib, g, cb, rr, ii, ri, ir);
    auto pack = [&](double (*dst)[64]) {
        int k = 0;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            dst[k++][lane] = rr[jj];
            if (AC && BC) dst[k++][lane] = ii[jj];
            if (BC) dst[k++][lane] = ri[jj];
            if (AC) dst[k++][lane] = ir[jj];
        }
    };
    if (wv > 0) pack(part[wv - 1]);
    __syncthreads();
    if (wv != 0) return;
#pragma unroll 1
    for (int w = 0; w < W - 1; ++w) {          // one wave's partials at a time (registers)
        int k = 0;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            rr[jj] += part[w][k++][lane];
            if (AC && BC) ii[jj] += part[w][k++][lane];
            if (BC) ri[jj] += part[w][k++][lane];
            if (AC) ir[jj] += part[w][k++][lane];
        }
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int p = cout[c * 16 + 4 * jj + g];
        if (p >= 0) {
            const double re = rr[jj] - ii[jj], im = ri[jj] + ir[jj];
            const int64_t o = (int64_t)p * 16 + q * 4 + r;
            cr[o] = alr * re - ali * im;
            if (ci) ci[o] = alr * im + ali * re;
        }
    }
}

// Below this many runs a product takes the split form (one run per
// workgroup): a wave per run would leave most of the 1,024 SIMDs idle.  Below
// kB4Split8Runs the runs are split over 8 waves instead of 4 (16 measured no
// faster on the 64-atom cluster).
constexpr int64_t kB4SplitRuns = 4096, kB4Split8Runs = 1024;

bool b4_split_form(int64_t nch) { return nch < kB4SplitRuns; }

template <bool AC, bool BC, int OB>
static void launch_b4j(hipStream_t s, const SpgemmArgs &a)
{
    RT_CHECK(a.nj == 16, RTDM_E_ARG, "b = 4 row runs hold 16 outputs");
    if (a.nch < kB4Split8Runs) {
        hipLaunchKernelGGL((k_spgemm_b4js<AC, BC, OB, 8>), dim3((unsigned)a.nch), dim3(512), 0, s, a.nch,
                           a.ch_off, a.ch_a, a.ch_b, a.ch_out, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,
                           a.alpha_im);
        return;
    }
    if (a.nch < kB4SplitRuns) {
        hipLaunchKernelGGL((k_spgemm_b4js<AC, BC, OB, 4>), dim3((unsigned)a.nch), dim3(256), 0, s, a.nch,
                           a.ch_off, a.ch_a, a.ch_b, a.ch_out, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,
                           a.alpha_im);
        return;
    }
    const int remap = b4_chunk();
    hipLaunchKernelGGL((k_spgemm_b4j<AC, BC, OB>), dim3(xcd_grid((a.nch + 3) / 4, remap)), dim3(256), 0, s,
                       a.nch, a.ch_off, a.ch_a, a.ch_b, a.ch_out, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,
                       a.alpha_im, remap);
}

template <bool AC, bool BC, int OB>
static void launch_b4w(hipStream_t s, const SpgemmArgs &a)
{
    hipLaunchKernelGGL((k_spgemm_b4w<AC, BC, OB>), dim3((unsigned)((a.nout + 63) / 64)), dim3(256), 0, s, a.nout,
                       a.off, a.trip, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re, a.alpha_im);
}

template <int SUB, bool AC, bool BC, int OA, int OB>
static void launch_b4(hipStream_t s, const SpgemmArgs &a)
{
    constexpr int OUT = 4 / SUB;
    const int64_t waves = (a.nout + OUT - 1) / OUT;
    hipLaunchKernelGGL((k_spgemm_b4<SUB, AC, BC, OA, OB>), dim3((unsigned)((waves + 3) / 4)), dim3(256),
                       0, s, a.nout, a.off, a.trip, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,
                       a.alpha_im);
}

template <bool AC, bool BC, int OA, int OB>
static void launch_split(hipStream_t s, const SpgemmArgs &a, dim3 g, dim3 t)
{
#define RT_SPLIT(B_, M_)                                                                         \
    hipLaunchKernelGGL((k_spgemm_split<B_, AC, BC, OA, OB, M_>), g, t, 0, s, a.nout, a.off, a.trip, \
                       a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re, a.alpha_im, a.maxabs)
    const int mode = a.precision == RTDM_PREC_FP16X2 ? 1 : 0;
    if (a.b == 13 && mode == 0) RT_SPLIT(13, 0);
    else if (a.b == 13) RT_SPLIT(13, 1);
    else if (mode == 0) RT_SPLIT(4, 0);
    else RT_SPLIT(4, 1);
#undef RT_SPLIT
}

template <bool AC, bool BC>
static void dispatch_ops(hipStream_t s, const SpgemmArgs &a, dim3 g, dim3 t)
{
#define RT_LAUNCH(OA, OB)                                                                        \
    do {                                                                                         \
        if (a.precision != RTDM_PREC_FP64 && a.b == 4 && OA == 0)                                \
            launch_b4x<AC, BC, OB>(s, a);                                                        \
        else if (a.precision == RTDM_PREC_BF16X3 || a.precision == RTDM_PREC_FP16X2)             \
            launch_split<AC, BC, OA, OB>(s, a, g, t);                                            \
        else if (a.precision == RTDM_PREC_FP32 && a.b == 13)                                     \
            hipLaunchKernelGGL((k_spgemm_kc<13, AC, BC, OA, OB, float>), g, t, 0, s, a.nout,     \
                               a.off, a.trip, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,    \
                               a.alpha_im);                                                      \
        else if (a.precision == RTDM_PREC_FP32 && a.b >= 4)                                      \
            hipLaunchKernelGGL((k_spgemm_kc<4, AC, BC, OA, OB, float>), g, t, 0, s, a.nout,      \
                               a.off, a.trip, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,    \
                               a.alpha_im);                                                      \
        else if (a.b == 4 && OA == 0 && a.nch > 0)                                               \
            launch_b4j<AC, BC, OB>(s, a);                                                        \
        else if (a.b == 4 && OA == 0)                                                            \
            launch_b4w<AC, BC, OB>(s, a);                                                        \
        else if (a.b == 4)                                                                       \
            launch_b4<(AC && BC) ? 4 : ((AC || BC) ? 2 : 1), AC, BC, OA, OB>(s, a);              \
        else if (a.b == 13)                                                                      \
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

// Step products with a column-major copy of the left operand (op(A)[r][m] at
// m*B + r) and a right operand whose op(B)[m][r] sits at m*B + r (row-major
// B, or the column-major copy of a matrix used conjugate-transposed).
template <bool AC, bool BC, int CJB, int LC>
static void launch_cm(hipStream_t s, const SpgemmArgs &a, dim3 g, dim3 t)
{
    {
        const int wpb = a.wpb;
        const int remap = xcd_chunk_wg(wpb);
        const unsigned grid = xcd_grid((a.nout + wpb - 1) / wpb, remap);
#define RT_Q4(W, T)                                                                               \
    hipLaunchKernelGGL((k_spgemm_q4<13, AC, BC, 0, CJB, LC, W, T>), dim3(grid), dim3(64 * W), 0, s, \
                       a.nout, a.off, a.trip, a.ar, a.ai, a.br, a.bi, a.cr, a.ci, a.alpha_re,       \
                       a.alpha_im, a.zero, a.order, remap)
        if (a.precision == RTDM_PREC_FP32) {
            if (wpb == 16) RT_Q4(16, float);
            else if (wpb == 8) RT_Q4(8, float);
            else RT_Q4(4, float);
        } else {
            if (wpb == 16) RT_Q4(16, double);
            else if (wpb == 8) RT_Q4(8, double);
            else RT_Q4(4, double);
        }
#undef RT_Q4
    }
}

// Row-run kernel (k_spgemm_q4j): runs of 2, 3 or 4 outputs, or 8 for real operands.
template <bool AC, bool BC, int CJB, int LC>
static void launch_cmj(hipStream_t s, const SpgemmArgs &a)
{
    const int remap = xcd_chunk();
    const unsigned grid = xcd_grid((a.nch + 3) / 4, remap);
    const bool f32 = a.precision == RTDM_PREC_FP32;
#define RT_Q4J_W(NJ, T, W)                                                                       \
    hipLaunchKernelGGL((k_spgemm_q4j<13, AC, BC, CJB, LC, NJ, T, W>), dim3(grid), dim3(256), 0, s,   \
                       a.nch,                                                                         \
                       a.ch_off, a.ch_a, a.ch_b, a.ch_out, a.ar, a.ai, a.br, a.bi, a.cr, a.ci,        \
                       a.alpha_re, a.alpha_im, a.zero, a.ch_order, remap, a.ch_seg)
#define RT_Q4J(NJ, T) RT_Q4J_W(NJ, T, 1)
    if (a.nj == 2) {
        // complex runs of 2 compiled for at least 4 waves per SIMD (at most 128
        // registers): 4 % faster than the compiler's 3; real runs lose 12 % so
        if (f32) RT_Q4J(2, float);
        else RT_Q4J_W(2, double, (AC && BC) ? 4 : 1);
    } else if (a.nj == 3) {
        if (f32) RT_Q4J(3, float);
        else RT_Q4J_W(3, double, (AC && BC) ? 4 : 1);
    } else if (a.nj == 4) {
        if (f32) RT_Q4J(4, float);
        else RT_Q4J(4, double);
    } else {
        if constexpr (!AC && !BC) {
            RT_CHECK(a.nj == 8, RTDM_E_ARG, "row runs of 2, 3, 4 or 8 outputs");
            if (f32) RT_Q4J(8, float);
            else RT_Q4J(8, double);
        } else {
            RT_CHECK(false, RTDM_E_ARG, "row runs of complex products hold 2, 3 or 4 outputs");
        }
    }
#undef RT_Q4J
#undef RT_Q4J_W
}

void launch_spgemm_cm(hipStream_t s, const SpgemmArgs &a, int conj_b, int out_col_major)
{
    if (a.nout == 0) return;
    RT_CHECK(a.b == 13 && (a.precision == RTDM_PREC_FP64 || a.precision == RTDM_PREC_FP32), RTDM_E_UNSUPPORTED,
             "column-major step products need b = 13 and FP64 or FP32");
    const dim3 g((unsigned)((a.nout + 3) / 4)), t(256);
    const bool ac = a.ai != nullptr, bc = a.bi != nullptr;
#define RT_CM(AC_, BC_)                                                            \
    do {                                                                           \
        if (a.nch > 0) {                                                           \
            if (conj_b && out_col_major) launch_cmj<AC_, BC_, 1, 1>(s, a);         \
            else if (conj_b) launch_cmj<AC_, BC_, 1, 0>(s, a);                     \
            else if (out_col_major) launch_cmj<AC_, BC_, 0, 1>(s, a);              \
            else launch_cmj<AC_, BC_, 0, 0>(s, a);                                 \
        } else if (conj_b && out_col_major) launch_cm<AC_, BC_, 1, 1>(s, a, g, t); \
        else if (conj_b) launch_cm<AC_, BC_, 1, 0>(s, a, g, t);                    \
        else if (out_col_major) launch_cm<AC_, BC_, 0, 1>(s, a, g, t);             \
        else launch_cm<AC_, BC_, 0, 0>(s, a, g, t);                                \
    } while (0)
    if (ac && bc) RT_CM(true, true);
    else if (ac) RT_CM(true, false);
    else if (bc) RT_CM(false, true);
    else RT_CM(false, false);
#undef RT_CM
    RT_HIP(hipGetLastError());
}


// FP32 variant of k_spgemm_q4 for real operands (the Taylor-term products of
// the reduced-precision form): column-major FP32 left operand, row-major FP32
// right operand, v_mfma_f32_16x16x4_f32 with FP32 accumulation, FP32 output
// scaled by alpha.  Same four-triple grouping, order and XCD mapping.
template <int B, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_spgemm_q4r32(
    int64_t nout, const int64_t *__restrict__ off, const int2 *__restrict__ trip,
    const float *__restrict__ a, const float *__restrict__ b, float *__restrict__ cout, float alpha,
    const float *__restrict__ zero, const int32_t *__restrict__ order)
{
    constexpr int BB = B * B;
    const int lane = threadIdx.x & 63;
    const int64_t w = xcd_block((nout + WPB - 1) / WPB) * WPB + (threadIdx.x >> 6);
    if (w >= nout) return;                     // uniform across the wave
    const int64_t c = order ? (int64_t)order[w] : w;
    const int r = lane & 15, q = lane >> 4;
    const bool rv = r < B;
    const int64_t t0 = off[c];
    const int nt = (int)(off[c + 1] - t0);
    typedef Mfma16<float>::acc_t acc_t;
    acc_t acc = {0, 0, 0, 0};
    for (int g = 0; g < nt; g += 4) {
        const float *pa = zero, *pb = zero;
        if (rv && g + q < nt) {
            const int2 ab = trip[t0 + g + q];
            pa = a + (int64_t)ab.x * BB + r;
            pb = b + (int64_t)ab.y * BB + r;
        }
#pragma unroll
        for (int st = 0; st < B; ++st) acc = Mfma16<float>::step(pa[st * B], pb[st * B], acc);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = Mfma16<float>::row(e, q), col = r;
        if (row < B && col < B) cout[c * BB + row * B + col] = alpha * acc[e];
    }
}

// Row-run form of k_spgemm_q4r32 (the dataflow of k_spgemm_q4j on FP32
// storage): NJ outputs of one row per wave, each loaded left-operand element
// feeding NJ FP32 MFMAs.
typedef __attribute__((address_space(1))) const float gfloat;
template <int B, int NJ>
__global__ __launch_bounds__(256) void k_spgemm_q4jr32(
    int64_t nch, const int64_t *__restrict__ off, const int32_t *__restrict__ ea,
    const int32_t *__restrict__ eb, const int32_t *__restrict__ cidx, const float *__restrict__ a,
    const float *__restrict__ b, float *__restrict__ cout, float alpha, const float *__restrict__ zero,
    const int32_t *__restrict__ order, int remap, const int32_t *__restrict__ seg)
{
    constexpr int BB = B * B;
    const int lane = threadIdx.x & 63;
    const int64_t w = xcd_block((nch + 3) / 4, remap) * 4 + (threadIdx.x >> 6);
    if (w >= nch) return;                      // uniform across the wave
    const int64_t c = order ? (int64_t)order[w] : w;
    const int r = lane & 15, q = lane >> 4;
    const bool rv = r < B;
    const int64_t e0 = off[c];
    const int ne = (int)(off[c + 1] - e0);
    typedef Mfma16<float>::acc_t acc_t;
    acc_t acc[NJ];
#pragma unroll
    for (int t = 0; t < NJ; ++t) acc[t] = acc_t{0, 0, 0, 0};
    const gfloat *gz = (const gfloat *)zero;
    // entries [gb, ge); output t's products only where bit t of ACT is set (segments as in k_spgemm_q4j)
    auto groups = [&](int gb, int ge, auto act) {
        constexpr int ACT = decltype(act)::value;
        for (int g = gb; g < ge; g += 4) {
            const gfloat *pa = gz;
            const gfloat *pb[NJ];
#pragma unroll
            for (int t = 0; t < NJ; ++t) pb[t] = gz;
            if (rv && g + q < ge) {
                const int64_t e = e0 + g + q;
                pa = (const gfloat *)(a + (int64_t)ea[e] * BB + r);
#pragma unroll
                for (int t = 0; t < NJ; ++t) {
                    if (!((ACT >> t) & 1)) continue;
                    const int kb = eb[e * NJ + t];
                    if (kb >= 0) pb[t] = (const gfloat *)(b + (int64_t)kb * BB + r);
                }
            }
#pragma unroll
            for (int st = 0; st < B; ++st) {
                const float xa = pa[st * B];
#pragma unroll
                for (int t = 0; t < NJ; ++t)
                    if ((ACT >> t) & 1) acc[t] = Mfma16<float>::step(xa, pb[t][st * B], acc[t]);
            }
        }
    };
    constexpr int ALL = (1 << NJ) - 1;
    if constexpr (NJ == 2) {
        if (seg) {
            const int nf = seg[2 * c], n0 = seg[2 * c + 1];   // uniform across the wave
            groups(0, nf, std::integral_constant<int, 3>());
            groups(nf, nf + n0, std::integral_constant<int, 1>());
            groups(nf + n0, ne, std::integral_constant<int, 2>());
        } else {
            groups(0, ne, std::integral_constant<int, ALL>());
        }
    } else {
        groups(0, ne, std::integral_constant<int, ALL>());
    }
#pragma unroll
    for (int t = 0; t < NJ; ++t) {
        const int p = cidx[c * NJ + t];
        if (p < 0) continue;                   // uniform: a short run
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = Mfma16<float>::row(e, q), col = r;
            if (row < B && col < B) cout[(int64_t)p * BB + row * B + col] = alpha * acc[t][e];
        }
    }
}

// Real FP32-storage b = 4 product (the late Taylor terms of the fp32_taylor
// form): FP32 row-major blocks, v_mfma_f32_4x4x1_16b with FP32 accumulation,
// FP32 output scaled by alpha; lane 4 blk + r holds row r of A_blk and
// column r of B_blk.  RUNS: one row run of 16 outputs per wave (entries
// shared by all blocks, b = 4 slot order); otherwise 16 consecutive outputs
// per wave, each with its own triple list.
template <bool RUNS>
__global__ __launch_bounds__(256) void k_spgemm_b4r32(
    int64_t n, const int64_t *__restrict__ off, const int2 *__restrict__ trip, const int32_t *__restrict__ ea,
    const int32_t *__restrict__ eb, const int32_t *__restrict__ rout, const float *__restrict__ a,
    const float *__restrict__ b, float *__restrict__ c32, float alpha)
{
    const int lane = threadIdx.x & 63;
    const int blk = lane >> 2, r = lane & 3;
    const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t c0 = RUNS ? wv : wv * 16;
    if (c0 >= n) return;                       // uniform across the wave
    const int64_t c = RUNS ? (int64_t)rout[wv * 16 + blk] : c0 + blk;
    const bool live = RUNS ? c >= 0 : c < n;
    const int64_t t0 = RUNS ? off[wv] : (live ? off[c] : 0);
    const int nt = RUNS ? (int)(off[wv + 1] - t0) : (live ? (int)(off[c + 1] - t0) : 0);
    int ntmax = nt;
    if (!RUNS) {
#pragma unroll
        for (int o = 4; o < 64; o <<= 1) ntmax = max(ntmax, __shfl_xor(ntmax, o, 64));
    }
    const int slot = (blk & 3) * 4 + (blk >> 2);
    f32x4 h = {0, 0, 0, 0};
    auto load_ops = [&](int2 ab, float (&xa)[4], float (&xb)[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) xa[k] = xb[k] = 0.0f;
        if (ab.y >= 0) {
            const f32x4 ar4 = *reinterpret_cast<const f32x4 *>(a + (int64_t)ab.x * 16 + r * 4);   // A[r][0..3]
            const int64_t pb = (int64_t)ab.y * 16 + r;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                xa[k] = ar4[k];
                xb[k] = b[pb + k * 4];                                                         // B[k][r]
            }
        }
    };
    if constexpr (RUNS) {
        // software pipeline as in b4_run_entries: indices two entries ahead,
        // operands one entry ahead, products in entry order
        auto load_idx = [&](int t) { return make_int2(ea[t0 + t], eb[(t0 + t) * 16 + slot]); };
        if (nt > 0) {
            float xa[4], xb[4];
            int2 ab_n = make_int2(0, -1);
            const int2 ab0 = load_idx(0);
            if (1 < nt) ab_n = load_idx(1);
            load_ops(ab0, xa, xb);
            for (int t = 0; t < nt; ++t) {
                int2 ab_nn = make_int2(0, -1);
                if (t + 2 < nt) ab_nn = load_idx(t + 2);
                float na[4] = {0, 0, 0, 0}, nb[4] = {0, 0, 0, 0};
                if (t + 1 < nt) load_ops(ab_n, na, nb);
#pragma unroll
                for (int k = 0; k < 4; ++k) h = __builtin_amdgcn_mfma_f32_4x4x1f32(xa[k], xb[k], h, 0, 0, 0);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    xa[k] = na[k];
                    xb[k] = nb[k];
                }
                ab_n = ab_nn;
            }
        }
    } else {
        for (int t = 0; t < ntmax; ++t) {
            const int2 ab = t < nt ? trip[t0 + t] : make_int2(0, -1);
            float xa[4], xb[4];
            load_ops(ab, xa, xb);
#pragma unroll
            for (int k = 0; k < 4; ++k) h = __builtin_amdgcn_mfma_f32_4x4x1f32(xa[k], xb[k], h, 0, 0, 0);
        }
    }
    if (!live) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) c32[c * 16 + e * 4 + r] = alpha * h[e];
}

// BF16 x 2 storage of b = 4 blocks for the BF16x3 late Taylor terms: x =
// hi + lo with the split of the register-split kernels (Split4<0>: round to
// FP32, hi its BF16 rounding, lo that of the remainder).  Block p takes 32
// values, its 16 hi parts then its 16 lo parts (64 bytes, one memory sector
// like an FP32 block); `transpose` stores each block transposed, so that
// column r of a right operand is four contiguous values.
__global__ void k_to_bf16x2(int64_t n, int transpose, const double *__restrict__ in, short *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int w = (int)(e & 15);
        const int64_t o = (e >> 4) * 32 + (transpose ? (w & 3) * 4 + (w >> 2) : w);
        short h, l;
        Split4<0>::split(in[e], 1.0f, h, l);
        out[o] = h;
        out[o + 16] = l;
    }
}

void launch_to_bf16x2(hipStream_t s, int64_t nblocks, int transpose, const double *in, short *out)
{
    const int64_t n = nblocks * 16;
    if (n == 0) return;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_to_bf16x2, dim3((unsigned)g), dim3(256), 0, s, n, transpose, in, out);
    RT_HIP(hipGetLastError());
}

// BF16x3 late Taylor term at b = 4 over row runs of 16 outputs, operands
// stored split (launch_to_bf16x2: A row-major, tau transposed): one wave per
// run, lane 4 blk + r holding row r of the entry's A block and column r of
// output blk's B block as four BF16 values per part (8-byte loads), three
// v_mfma_f32_4x4x4_16b_bf16 per entry (hi hi, then hi lo and lo hi into a
// second accumulator).  The result tau = alpha (h + m) is added into the FP64
// plane u (u += u_sign tau: the propagator's sum) and, when c16 is set,
// stored split and transposed as the next term's right operand.  The split,
// the products and their order per output are those of the register-split
// kernel (k_spgemm_b4x<..., 1, true>); this one moves half of its operand
// bytes per triple (two 16-bit values instead of one FP64 per element).
__global__ __launch_bounds__(256) void k_spgemm_b4r16(
    int64_t nch, const int64_t *__restrict__ off, const int32_t *__restrict__ ea, const int32_t *__restrict__ eb,
    const int32_t *__restrict__ rout, const short *__restrict__ a16, const short *__restrict__ b16,
    short *__restrict__ c16, double alpha, double *__restrict__ u, double u_sign)
{
    typedef short v4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const int blk = lane >> 2, r = lane & 3;
    const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wv >= nch) return;                     // uniform across the wave
    const int64_t c = rout[wv * 16 + blk];
    const int64_t t0 = off[wv];
    const int nt = (int)(off[wv + 1] - t0);
    const int slot = (blk & 3) * 4 + (blk >> 2);
    f32x4 h = {0, 0, 0, 0}, m = {0, 0, 0, 0};
    struct Ops {
        v4 ah, al, bh, bl;
    };
    auto load_idx = [&](int t) { return make_int2(ea[t0 + t], eb[(t0 + t) * 16 + slot]); };
    auto load_ops = [&](int2 ab, Ops &o) {
        o.ah = o.al = o.bh = o.bl = v4{0, 0, 0, 0};
        if (ab.y >= 0) {
            const short *pa = a16 + (int64_t)ab.x * 32 + r * 4, *pb = b16 + (int64_t)ab.y * 32 + r * 4;
            o.ah = *reinterpret_cast<const v4 *>(pa);        // A[r][0..3]
            o.al = *reinterpret_cast<const v4 *>(pa + 16);
            o.bh = *reinterpret_cast<const v4 *>(pb);        // B[0..3][r]
            o.bl = *reinterpret_cast<const v4 *>(pb + 16);
        }
    };
    if (nt > 0) {
        // software pipeline as in b4_run_entries: indices two entries ahead, operands one
        Ops cur, nxt;
        int2 ab_n = make_int2(0, -1);
        const int2 ab0 = load_idx(0);
        if (1 < nt) ab_n = load_idx(1);
        load_ops(ab0, cur);
        for (int t = 0; t < nt; ++t) {
            int2 ab_nn = make_int2(0, -1);
            if (t + 2 < nt) ab_nn = load_idx(t + 2);
            if (t + 1 < nt) load_ops(ab_n, nxt);
            h = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(cur.ah, cur.bh, h, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(cur.ah, cur.bl, m, 0, 0, 0);
            m = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(cur.al, cur.bh, m, 0, 0, 0);
            cur = nxt;
            ab_n = ab_nn;
        }
    }
    if (c < 0) return;
    v4 sh, sl;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double v = alpha * ((double)h[e] + 1.0 * (double)m[e]);
        const int64_t o = c * 16 + e * 4 + r;
        u[o] = u[o] + u_sign * v;
        short hh, ll;
        Split4<0>::split(v, 1.0f, hh, ll);
        sh[e] = hh;
        sl[e] = ll;
    }
    if (c16) {
        *reinterpret_cast<v4 *>(c16 + c * 32 + r * 4) = sh;        // transposed: column r of the block
        *reinterpret_cast<v4 *>(c16 + c * 32 + 16 + r * 4) = sl;
    }
}

void launch_spgemm_r16(hipStream_t s, const SpgemmArgs &a, const short *a16, const short *b16, short *c16,
                       double *u, double u_sign)
{
    RT_CHECK(a.b == 4 && a.nch > 0 && a.nj == 16, RTDM_E_ARG, "split BF16 Taylor terms need b = 4 row runs of 16");
    hipLaunchKernelGGL(k_spgemm_b4r16, dim3((unsigned)((a.nch + 3) / 4)), dim3(256), 0, s, a.nch, a.ch_off, a.ch_a,
                       a.ch_b, a.ch_out, a16, b16, c16, a.alpha_re, u, u_sign);
    RT_HIP(hipGetLastError());
}

void launch_spgemm_r32(hipStream_t s, const SpgemmArgs &a, const float *a32, const float *b32, float *c32,
                       const float *zero32)
{
    if (a.nout == 0) return;
    RT_CHECK(a.b == 13 || a.b == 4, RTDM_E_UNSUPPORTED, "FP32 step products need b = 4 or 13");
    if (a.b == 4) {
        if (a.nch > 0) {
            RT_CHECK(a.nj == 16, RTDM_E_ARG, "b = 4 row runs hold 16 outputs");
            hipLaunchKernelGGL(k_spgemm_b4r32<true>, dim3((unsigned)((a.nch + 3) / 4)), dim3(256), 0, s, a.nch,
                               a.ch_off, nullptr, a.ch_a, a.ch_b, a.ch_out, a32, b32, c32, (float)a.alpha_re);
        } else {
            hipLaunchKernelGGL(k_spgemm_b4r32<false>, dim3((unsigned)((a.nout + 63) / 64)), dim3(256), 0, s,
                               a.nout, a.off, a.trip, nullptr, nullptr, nullptr, a32, b32, c32, (float)a.alpha_re);
        }
        RT_HIP(hipGetLastError());
        return;
    }
    if (a.nch > 0) {
        const int remap = xcd_chunk();
        const unsigned grid = xcd_grid((a.nch + 3) / 4, remap);
#define RT_R32J(NJ)                                                                                     \
    hipLaunchKernelGGL((k_spgemm_q4jr32<13, NJ>), dim3(grid), dim3(256), 0, s, a.nch, a.ch_off, a.ch_a, \
                       a.ch_b, a.ch_out, a32, b32, c32, (float)a.alpha_re, zero32, a.ch_order, remap, a.ch_seg)
        if (a.nj == 2) RT_R32J(2);
        else if (a.nj == 3) RT_R32J(3);
        else if (a.nj == 4) RT_R32J(4);
        else {
            RT_CHECK(a.nj == 8, RTDM_E_ARG, "row runs of 2, 4 or 8 outputs");
            RT_R32J(8);
        }
#undef RT_R32J
        RT_HIP(hipGetLastError());
        return;
    }
    const int wpb = a.wpb;
    const unsigned grid = xcd_grid((a.nout + wpb - 1) / wpb);
#define RT_R32(W)                                                                                  \
    hipLaunchKernelGGL((k_spgemm_q4r32<13, W>), dim3(grid), dim3(64 * W), 0, s, a.nout, a.off, a.trip, \
                       a32, b32, c32, (float)a.alpha_re, zero32, a.order)
    if (wpb == 16) RT_R32(16);
    else if (wpb == 8) RT_R32(8);
    else RT_R32(4);
#undef RT_R32
    RT_HIP(hipGetLastError());
}

void launch_spgemm(hipStream_t s, const SpgemmArgs &a)
{
    if (a.nout == 0) return;
    RT_CHECK(a.b >= 1 && a.b <= 16, RTDM_E_UNSUPPORTED, "block size must be 1..16");
    RT_CHECK(a.precision == RTDM_PREC_FP64 || (a.b == 4 || a.b == 13), RTDM_E_UNSUPPORTED,
             "reduced-precision products need b = 4 or 13");
    RT_CHECK(a.precision != RTDM_PREC_FP16X2 || a.maxabs, RTDM_E_ARG, "FP16 split products need operand maxima");
    const dim3 g((unsigned)((a.nout + 3) / 4)), t(256);
    const bool ac = a.ai != nullptr, bc = a.bi != nullptr;
    if (ac && bc) dispatch_ops<true, true>(s, a, g, t);
    else if (ac) dispatch_ops<true, false>(s, a, g, t);
    else if (bc) dispatch_ops<false, true>(s, a, g, t);
    else dispatch_ops<false, false>(s, a, g, t);
    RT_HIP(hipGetLastError());
}

}  // namespace rtdm

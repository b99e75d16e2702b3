// C ABI of the truncated block-sparse RT-TDDFT propagation library (rtdm.h).
//
// Host side: atom-pair neighbour lists (cell lists), symbolic schedules of
// every truncated product, device storage of the blocked matrices (real and
// imaginary parts in separate planes, blocks b*b row-major in pattern order),
// the truncated Hotelling iteration (Sec. V.A), the exponential-midpoint step
// with a Taylor propagator (Sec. II.A, Eq. EM, Eq. matrix_exp, Sec. IV.B) and
// the observables (Sec. II.B dipole, Sec. IV charge and unitarity).
//
// The propagator uses that S, H and hence X ~ S^-1 and A = X H are real (the
// paper's support functions and Hamiltonian are real): then
// T_n = (-i dt / n) A T_{n-1} = (-i)^n tau_n with real tau_n = (dt/n) A tau_{n-1},
// so U = sum_n T_n has Re U = tau_0 - tau_2 + tau_4 - ... and
// Im U = -tau_1 + tau_3 - tau_5 + ..., and every product that builds U is a
// real block product.  The values are the ones the complex recursion gives
// (the other part of every term is exactly zero).
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <random>
#include <tuple>
#include <vector>

#include "internal.h"

namespace rtdm {

thread_local DevMem *g_devmem = nullptr;

void *devmem_alloc(DBufBase *b, size_t bytes)
{
    DevMem *m = g_devmem;
    void *p = nullptr;
    if (m && m->base) {
        const size_t off = devmem_align(m->used);
        RT_CHECK(off + bytes <= m->cap, RTDM_E_OOM,
                 "bound workspace exhausted: " + std::to_string(bytes) + " more bytes needed");
        p = m->base + off;
        m->used = off + bytes;
        b->in_ws = true;
    } else if (m && m->ext_alloc) {
        p = m->ext_alloc(bytes, m->ext_user);
        RT_CHECK(p, RTDM_E_OOM, "the caller's allocator refused " + std::to_string(bytes) + " bytes");
        RT_CHECK((reinterpret_cast<uintptr_t>(p) & 255) == 0, RTDM_E_ARG,
                 "the caller's allocator returned memory that is not 256-byte aligned");
        b->in_ws = false;
        b->ext = true;
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(RTDM_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        b->in_ws = false;
        b->ext = false;
    }
    b->mem = m;
    b->nbytes = bytes;
    if (m) m->bufs.insert(b);
    return p;
}

void devmem_free(DBufBase *b, void *p)
{
    DevMem *m = b->mem;
    if (b->in_ws) {
        // the most recent slice (a temporary of the current call) is given back
        if (m && static_cast<char *>(p) + b->nbytes == m->base + m->used)
            m->used = (size_t)(static_cast<char *>(p) - m->base);
    } else if (b->ext) {
        // the caller's allocator may hand the memory out again at once (a
        // caching allocator does, to work ordered on another stream): let every
        // kernel that may still use it finish first
        (void)hipDeviceSynchronize();
        m->ext_free(p, m->ext_user);
    } else {
        (void)hipFree(p);
    }
    if (m) m->bufs.erase(b);
    b->mem = nullptr;
    b->nbytes = 0;
    b->in_ws = false;
    b->ext = false;
}

void devmem_moved(DBufBase *from, DBufBase *to)
{
    if (!to->mem) return;
    to->mem->bufs.erase(from);
    to->mem->bufs.insert(to);
}

}  // namespace rtdm

namespace {
// Makes a context's registry the current one for the duration of an API call.
struct DevMemScope {
    rtdm::DevMem *saved;
    explicit DevMemScope(rtdm::DevMem *m) : saved(rtdm::g_devmem) { rtdm::g_devmem = m; }
    ~DevMemScope() { rtdm::g_devmem = saved; }
};
constexpr size_t kWorkspaceReserve = size_t(64) << 20;   // per-call temporaries, trace growth
}  // namespace

using namespace rtdm;

namespace {

enum Range { R_HS = 0, R_P = 1, R_K = 2 };

struct Pattern {
    double R = 0.0;
    int64_t n = 0, nnzb = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col, rowof, trans, diag;
    DBuf<int64_t> d_rowptr;
    DBuf<int32_t> d_col, d_rowof, d_trans, d_diag;
};

struct Mat {
    int pat = -1;
    bool cplx = false;
    DBuf<double> re, im;
};

// Row runs of one schedule for one run length nj (see build_runs).
struct Runs {
    int nj = 0;
    int64_t nch = 0;
    DBuf<int64_t> off;
    DBuf<int32_t> a, b, out, order;
    DBuf<int32_t> seg;               // runs of 2 at b = 13: segment sizes (SpgemmArgs::ch_seg)
    std::vector<int32_t> row, col;   // row and first column of each run
};

struct Sched {
    int64_t nout = 0, ntrip = 0;
    DBuf<int64_t> off;
    DBuf<int2> trip;
    DBuf<int32_t> order;   // processing order of the output blocks (row tiles, then columns)
    // row runs of this schedule (SpgemmArgs::ch_*), by run length
    std::map<int, std::unique_ptr<Runs>> runs;
};

// Processing order of the output blocks of pattern C: rows are cut into
// tiles of `tile_i` consecutive atoms and columns into tiles of `tile_j`
// consecutive atoms; a row tile is processed column tile by column tile, and
// inside a column tile column by column, row by row.  Consecutive outputs then
// share their right-operand blocks (same column), and the left- and
// right-operand blocks of one (row tile, column tile) pair stay in L2 while
// its outputs run.
std::vector<int32_t> tile_order(const Pattern &C, int tile_i, int tile_j)
{
    std::vector<int32_t> order;
    order.reserve(C.nnzb);
    struct E { int32_t jt, j, p; };
    std::vector<E> buf;
    for (int64_t i0 = 0; i0 < C.n; i0 += tile_i) {
        const int64_t i1 = std::min<int64_t>(C.n, i0 + tile_i);
        buf.clear();
        for (int64_t p = C.rowptr[i0]; p < C.rowptr[i1]; ++p)
            buf.push_back({C.col[p] / tile_j, C.col[p], (int32_t)p});
        std::stable_sort(buf.begin(), buf.end(), [](const E &x, const E &y) {
            return x.jt != y.jt ? x.jt < y.jt : x.j < y.j;
        });
        for (auto &e : buf) order.push_back(e.p);
    }
    return order;
}



// Processing order of row runs: rows in tiles of `tile_i` atoms; inside a
// tile by first column, then row (the order of tile_order for single outputs).
std::vector<int32_t> run_order(const Runs &R, int tile_i)
{
    std::vector<int32_t> ord(R.nch);
    for (int64_t u = 0; u < R.nch; ++u) ord[u] = (int32_t)u;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
        const int32_t tx = R.row[x] / tile_i, ty = R.row[y] / tile_i;
        return tx != ty ? tx < ty : R.col[x] < R.col[y];
    });
    return ord;
}

constexpr size_t kRunReserve = size_t(16) << 30;   // device memory row runs leave free

// Row runs of schedule S for op(A) = A: the outputs of each row of C cut into
// runs of nj consecutive columns; the entries of a run are the k of row i of
// A used by any of its outputs, each with op(A)_ik and the op(B)_kj block of
// every output (-1: no triple for k).  Built on the GPU (k_run_sym); inter4
// stores the b = 4 kernel's slot order.
bool build_runs(Sched &S, const Pattern &A, const Pattern &B, const Pattern &C, int op_b, int nj, int inter4,
                int tile_i)
{
    if (S.runs.count(nj)) return false;
    auto R = std::make_unique<Runs>();
    std::vector<int64_t> p0s;
    for (int64_t i = 0; i < C.n; ++i)
        for (int64_t p0 = C.rowptr[i]; p0 < C.rowptr[i + 1]; p0 += nj) {
            R->row.push_back((int32_t)i);
            R->col.push_back(C.col[p0]);
            p0s.push_back(p0);
        }
    R->nj = nj;
    R->nch = (int64_t)R->row.size();
    const int64_t nch = R->nch;
    DBuf<int32_t> d_row;
    DBuf<int64_t> d_p0, cnt;
    d_row.alloc(std::max<int64_t>(nch, 1));
    d_p0.alloc(std::max<int64_t>(nch, 1));
    cnt.alloc(std::max<int64_t>(nch, 1));
    // runs of 2 (b = 13) are stored in segments: entries feeding both outputs, then one
    const bool segmented = nj == 2 && !inter4;
    if (segmented) R->seg.alloc(std::max<int64_t>(2 * nch, 2));
    std::vector<int64_t> off(nch + 1, 0);
    if (nch) {
        RT_HIP(hipMemcpy(d_row.p, R->row.data(), nch * sizeof(int32_t), hipMemcpyHostToDevice));
        RT_HIP(hipMemcpy(d_p0.p, p0s.data(), nch * sizeof(int64_t), hipMemcpyHostToDevice));
        launch_run_count(nullptr, nch, d_row.p, d_p0.p, C.d_rowptr.p, C.d_col.p, A.d_rowptr.p, A.d_col.p,
                         B.d_rowptr.p, B.d_col.p, nj, cnt.p, segmented ? R->seg.p : nullptr);
        RT_HIP(hipMemcpy(off.data() + 1, cnt.p, nch * sizeof(int64_t), hipMemcpyDeviceToHost));
        for (int64_t u = 0; u < nch; ++u) off[u + 1] += off[u];
    }
    const int64_t ne = off[nch];
    {
        // optional: keep per-output lists where the runs would not leave room
        size_t free_b = 0, total_b = 0;
        RT_HIP(hipMemGetInfo(&free_b, &total_b));
        const double need = (double)ne * 4.0 * (1 + nj) + (double)nch * (8.0 + 4.0 * nj + 4.0);
        if (need + (double)kRunReserve > (double)free_b) return false;
    }
    R->off.alloc(nch + 1);
    R->a.alloc(std::max<int64_t>(ne, 1));
    R->b.alloc(std::max<int64_t>(ne * nj, 1));
    R->out.alloc(std::max<int64_t>(nch * nj, 1));
    R->order.alloc(std::max<int64_t>(nch, 1));
    RT_HIP(hipMemcpy(R->off.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    launch_run_fill(nullptr, nch, d_row.p, d_p0.p, C.d_rowptr.p, C.d_col.p, A.d_rowptr.p, A.d_col.p, B.d_rowptr.p,
                    B.d_col.p, B.d_trans.p, op_b, nj, inter4, R->off.p, R->a.p, R->b.p, R->out.p, segmented);
    const std::vector<int32_t> ord = run_order(*R, tile_i);
    if (!ord.empty())
        RT_HIP(hipMemcpy(R->order.p, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    RT_HIP(hipDeviceSynchronize());   // the temporaries above are freed on return
    S.runs.emplace(nj, std::move(R));
    return true;
}

struct TRec {
    int prod;
    int ev;
    double flops;
};

const char *kProdName[RTDM_PROD_COUNT] = {"XH", "AT", "UK", "WU", "SX", "UV", "ZX"};

// Learned starting guess: network parameters, Adam state, training samples.
struct MlpState {
    int b = 0, in = 0, out = 0;
    int64_t nw1 = 0, nb1 = 0, nw2 = 0, nb2 = 0, np = 0;
    DBuf<float> w, m, v, grad;
    DBuf<__half> w1h, w2h;
    int step = 0;
    bool ready = false;
    DBuf<float> ds_x, ds_t;
    int64_t ns = 0, cap = 0;
    DBuf<float> hid, y, dy, dh, sqerr, tx, tt;
    int64_t work_n = 0;
    DBuf<int32_t> idx;
    DBuf<double> dsum;
};

}  // namespace

struct rtdm_ctx {
    rtdm::DevMem mem;   // first member: destroyed after every buffer registered in it
    int device = 0;
    rtdm_options opt{};
    std::string err;

    int64_t n = 0;
    int b = 0;
    std::vector<double> xyz;
    DBuf<double> d_xyz;
    // per-atom block sizes: atoms with fewer than b functions are padded to b
    // (identity in S and X, zero elsewhere on the padded functions)
    bool mixed = false;
    std::vector<int32_t> nbf;
    DBuf<int32_t> d_nbf;
    int64_t n_pad = 0;          // padded functions in all

    double radius[3] = {0, 0, 0};
    bool ranges_set = false;
    std::vector<std::unique_ptr<Pattern>> pats;
    int range_pat[3] = {-1, -1, -1};

    Mat mats[RTDM_MAT_COUNT];
    Mat tau[2], Kn, Xn, Wh, V, Z;
    // Mulliken model: A0 = P(X H0), so that a step's A is A0 + X D (D diagonal)
    Mat A0;
    bool A0_valid = false;
    // b = 4, FP64 products over row runs: Uh = U^dagger stored as a matrix, so
    // that W U^dagger reads its right operand by rows of Uh (blocks of one row k
    // for the 16 outputs of a run) instead of by columns of U
    Mat Uh;
    bool Uh_on = false;
    bool u_copies_valid = false;   // Uc (b = 13) and Uh follow U
    // column-major block copies of the step's left operands (b = 13, FP64) and
    // of S for the inverse iteration
    Mat Xc, Ac, Uc, Wc, Sc;
    bool Xc_valid = false, W_in_cm = false;
    // FP32 copies for the reduced-precision Taylor terms (b = 13)
    DBuf<float> Ac32, tau32[2], zero32;
    DBuf<double> scratch;       // block inverse scratch and staging

    std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<Sched>> scheds;

    DBuf<int32_t> s_to_k, p_to_hs;
    DBuf<double> q_ref, q_a, q_b;
    double *q_cur = nullptr, *q_prev = nullptr;   // [n_kicks][n]: kick k's charges at + k n
    // kick sets (opt.n_kicks > 1): K of kick k is mats[K] (k = 0) or Kx[k - 1];
    // every kick shares S, H, X and U; the API reads kick kick_sel
    std::vector<Mat> Kx;
    int kick_sel = 0;
    bool q_ref_valid = false, charges_valid = false;

    bool uploaded[RTDM_MAT_COUNT] = {};
    bool X_valid = false, U_valid = false, s_norm_valid = false;
    double U_dt = 0.0;

    DBuf<double> obs;
    int64_t obs_cap = 0, obs_rows = 0;
    double t_now = 0.0;
    bool herm_valid = false;

    DBuf<double> partials, herm_sums, unit_sums, s_norm2, hot_sums, atom_max, obs_tmp, zero;

    int prec = RTDM_PREC_FP64;  // arithmetic of the products being issued
    MlpState mlp;
    DBuf<int32_t> hs_to_p, hs_iota;
    // device step state (trace row, steps in call; start time, dt) and groups
    DBuf<int64_t> step_st;
    DBuf<double> step_tt;
    bool obs_reset_pending = true;
    int64_t n_groups = 1;
    std::vector<int64_t> gptr;
    DBuf<int64_t> d_gptr;
    DBuf<int32_t> d_group;
    DBuf<double> obs_g, kick_g;
    // captured step
    hipStream_t gstream = nullptr;
    hipGraph_t graph = nullptr, graph_multi = nullptr;            // one step; opt.graph_steps steps
    hipGraphExec_t gexec = nullptr, gexec_multi = nullptr;
    bool capturing = false;
    uint64_t graph_epoch = 0;   // advances whenever captured steps of this context turn stale
    double graph_dt = 0.0;
    bool graph_rebuilds_u = false;
    // launch shape of the step products
    int wpb = 16, row_tile = 256;   // row tile of the b = 13 processing order (measured best with the XCD deal)
    int run_real = 2, run_cplx = 2;   // b = 13 step products: outputs per row run (1: single outputs)
    int run_b4 = 16;                  // b = 4 FP64 products: outputs per row run (1: single outputs)
    int inv_iters_total = 0, inv_fell_back = 0;
    // ETRS / Magnus work matrices and the self-consistent corrector's state
    Mat E1, E2, E3, A1, Kt;
    DBuf<double> q_c;           // q(t + dt) of the previous pass
    int64_t step_count = 0;     // steps since the last kick
    double trace_dt = 0.0;
    bool trace_dt_mixed = false;
    // external field E0 exp(-(t - t0)^2 / (2 sigma^2)); centres of the groups
    bool field_on = false;
    double field_E0[3] = {0.0, 0.0, 0.0}, field_t0 = 0.0, field_sigma = 1.0;
    DBuf<double> d_centre, d_centre_all;   // centres of the groups, of all atoms
    DBuf<double> f16_max;       // operand maxima of the FP16 split products
    bool timing = false;
    std::vector<hipEvent_t> events;
    std::vector<TRec> recs;
};

namespace {

void set_device(rtdm_ctx *c) { RT_HIP(hipSetDevice(c->device)); }

// Centroid of atoms i0 .. i1-1: each coordinate summed with compensation
// (Knuth's two-sum on every addition, the error terms accumulated in a second
// double), rounded once, then divided by the count.  For atom coordinates the
// error terms are far below the sum's last digit, so this is the correctly
// rounded sum, which every implementation that rounds the exact sum once
// also gets: the dipole about the centroid then does not depend on the
// summation order of the positions.
void exact_centre(const std::vector<double> &xyz, int64_t i0, int64_t i1, double out[3])
{
    for (int k = 0; k < 3; ++k) {
        double hi = 0.0, lo = 0.0;
        for (int64_t i = i0; i < i1; ++i) {
            const double x = xyz[3 * i + k], s = hi + x, bp = s - hi;
            lo += (hi - (s - bp)) + (x - bp);
            hi = s;
        }
        out[k] = (hi + lo) / (double)(i1 - i0);
    }
}

int n_kicks(const rtdm_ctx *c) { return c->opt.n_kicks; }
Mat &kmat(rtdm_ctx *c, int k) { return k == 0 ? c->mats[RTDM_MAT_K] : c->Kx[k - 1]; }
double *qcur(rtdm_ctx *c, int k) { return c->q_cur + (int64_t)k * c->n; }
double *qprev(rtdm_ctx *c, int k) { return c->q_prev + (int64_t)k * c->n; }
double *herm_of(rtdm_ctx *c, int k) { return c->herm_sums.p + 4 * k; }
double *obs_of(rtdm_ctx *c, int k) { return c->obs.p + (int64_t)k * c->obs_cap * 8; }
double *obs_g_of(rtdm_ctx *c, int k) { return c->obs_g.p + (int64_t)k * c->obs_cap * c->n_groups * 4; }

int slot_range(int m)
{
    switch (m) {
    case RTDM_MAT_S:
    case RTDM_MAT_H0:
    case RTDM_MAT_H: return R_HS;
    case RTDM_MAT_X:
    case RTDM_MAT_A:
    case RTDM_MAT_U: return R_P;
    default: return R_K;
    }
}

bool slot_complex(int m) { return m == RTDM_MAT_U || m == RTDM_MAT_K || m == RTDM_MAT_W; }

// Cut-off pattern of range R: cell lists of edge max(R, 1), kept pairs tested
// as dx*dx + dy*dy + dz*dz < R*R, self pairs always kept, rows ascending.
void build_pattern(Pattern &P, const std::vector<double> &xyz, int64_t n, double R)
{
    P.R = R;
    P.n = n;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], xyz[3 * i + a]);
            hi[a] = std::max(hi[a], xyz[3 * i + a]);
        }
    double edge = std::max(R, 1.0);
    int64_t nc[3];
    for (;;) {
        int64_t tot = 1;
        for (int a = 0; a < 3; ++a) {
            nc[a] = (int64_t)std::floor((hi[a] - lo[a]) / edge) + 1;
            tot *= nc[a];
        }
        if (tot <= 4 * n + 64) break;
        edge *= 1.5;
    }
    auto cell_of = [&](int64_t i, int a) {
        int64_t c = (int64_t)std::floor((xyz[3 * i + a] - lo[a]) / edge);
        return std::min(std::max<int64_t>(c, 0), nc[a] - 1);
    };
    const int64_t ncell = nc[0] * nc[1] * nc[2];
    std::vector<int64_t> head(ncell + 1, 0), order(n);
    std::vector<int64_t> cid(n);
    for (int64_t i = 0; i < n; ++i) {
        cid[i] = (cell_of(i, 0) * nc[1] + cell_of(i, 1)) * nc[2] + cell_of(i, 2);
        head[cid[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
    {
        std::vector<int64_t> fill(head.begin(), head.end() - 1);
        for (int64_t i = 0; i < n; ++i) order[fill[cid[i]]++] = i;
    }
    const double R2 = R * R;
    std::vector<std::vector<int32_t>> rows(n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t ci[3] = {cell_of(i, 0), cell_of(i, 1), cell_of(i, 2)};
        auto &row = rows[i];
        for (int64_t x = std::max<int64_t>(ci[0] - 1, 0); x <= std::min(ci[0] + 1, nc[0] - 1); ++x)
            for (int64_t y = std::max<int64_t>(ci[1] - 1, 0); y <= std::min(ci[1] + 1, nc[1] - 1); ++y)
                for (int64_t z = std::max<int64_t>(ci[2] - 1, 0); z <= std::min(ci[2] + 1, nc[2] - 1); ++z) {
                    const int64_t c = (x * nc[1] + y) * nc[2] + z;
                    for (int64_t q = head[c]; q < head[c + 1]; ++q) {
                        const int64_t j = order[q];
                        if (j == i) { row.push_back((int32_t)j); continue; }
                        const double dx = xyz[3 * i] - xyz[3 * j];
                        const double dy = xyz[3 * i + 1] - xyz[3 * j + 1];
                        const double dz = xyz[3 * i + 2] - xyz[3 * j + 2];
                        if (dx * dx + dy * dy + dz * dz < R2) row.push_back((int32_t)j);
                    }
                }
        std::sort(row.begin(), row.end());
    }
    P.rowptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) P.rowptr[i + 1] = P.rowptr[i] + (int64_t)rows[i].size();
    P.nnzb = P.rowptr[n];
    RT_CHECK(P.nnzb < (int64_t)INT32_MAX, RTDM_E_UNSUPPORTED, "more than 2^31 blocks in one pattern");
    P.col.resize(P.nnzb);
    P.rowof.resize(P.nnzb);
    for (int64_t i = 0; i < n; ++i) {
        std::copy(rows[i].begin(), rows[i].end(), P.col.begin() + P.rowptr[i]);
        std::fill(P.rowof.begin() + P.rowptr[i], P.rowof.begin() + P.rowptr[i + 1], (int32_t)i);
    }
    auto find = [&](int64_t i, int32_t j) -> int64_t {
        auto b0 = P.col.begin() + P.rowptr[i], b1 = P.col.begin() + P.rowptr[i + 1];
        auto it = std::lower_bound(b0, b1, j);
        return (it != b1 && *it == j) ? (int64_t)(it - P.col.begin()) : -1;
    };
    P.trans.resize(P.nnzb);
    P.diag.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = P.rowptr[i]; p < P.rowptr[i + 1]; ++p) {
            const int64_t t = find(P.col[p], (int32_t)i);
            RT_CHECK(t >= 0, RTDM_E_NUMERIC, "cut-off pattern is not symmetric");
            P.trans[p] = (int32_t)t;
        }
        P.diag[i] = (int32_t)find(i, (int32_t)i);
    }
    P.d_rowptr.alloc(n + 1);
    P.d_col.alloc(P.nnzb);
    P.d_rowof.alloc(P.nnzb);
    P.d_trans.alloc(P.nnzb);
    P.d_diag.alloc(n);
    RT_HIP(hipMemcpy(P.d_rowptr.p, P.rowptr.data(), P.d_rowptr.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(P.d_col.p, P.col.data(), P.d_col.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(P.d_rowof.p, P.rowof.data(), P.d_rowof.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(P.d_trans.p, P.trans.data(), P.d_trans.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(P.d_diag.p, P.diag.data(), P.d_diag.bytes(), hipMemcpyHostToDevice));
}

Pattern &pat_of(rtdm_ctx *c, int range) { return *c->pats[c->range_pat[range]]; }

int64_t elems(rtdm_ctx *c, const Mat &m) { return c->pats[m.pat]->nnzb * (int64_t)c->b * c->b; }

// Uninitialised matrix on the pattern (and with the planes) of `ref`.
void alloc_like(rtdm_ctx *c, Mat &m, const Mat &ref)
{
    m.pat = ref.pat;
    m.cplx = ref.cplx;
    const int64_t ne = c->pats[ref.pat]->nnzb * (int64_t)c->b * c->b;
    m.re.alloc(ne);
    if (ref.cplx) m.im.alloc(ne);
    else m.im.release();
}

void alloc_mat(rtdm_ctx *c, Mat &m, int range, bool cplx)
{
    m.pat = c->range_pat[range];
    m.cplx = cplx;
    const int64_t ne = pat_of(c, range).nnzb * (int64_t)c->b * c->b;
    m.re.alloc(ne);
    RT_HIP(hipMemset(m.re.p, 0, m.re.bytes()));
    if (cplx) {
        m.im.alloc(ne);
        RT_HIP(hipMemset(m.im.p, 0, m.im.bytes()));
    } else {
        m.im.release();
    }
}

void make_complex(rtdm_ctx *c, Mat &m, hipStream_t s)
{
    if (m.cplx) return;
    m.im.alloc(m.re.n);
    RT_HIP(hipMemsetAsync(m.im.p, 0, m.im.bytes(), s));
    m.cplx = true;
}

// (pattern A, pattern B, pattern C, op_a, op_b) of each product kind.
std::tuple<int, int, int, int, int> prod_key(rtdm_ctx *c, int prod)
{
    const int hs = c->range_pat[R_HS], p = c->range_pat[R_P], k = c->range_pat[R_K];
    switch (prod) {
    case RTDM_PROD_XH: return {p, hs, p, 0, 0};
    case RTDM_PROD_AT: return {p, p, p, 0, 0};
    case RTDM_PROD_UK: return {p, k, k, 0, 0};
    case RTDM_PROD_WU: return {k, p, k, 0, 1};
    case RTDM_PROD_SX: return {hs, p, p, 0, 0};
    case RTDM_PROD_UV: return {p, p, p, 1, 0};
    case RTDM_PROD_ZX: return {p, p, k, 0, 0};
    }
    throw Error(RTDM_E_ARG, "unknown product kind");
}

// W U^dagger with U^dagger stored (Uh): a plain product of patterns K, P -> K.
std::tuple<int, int, int, int, int> wuh_key(rtdm_ctx *c)
{
    return {c->range_pat[R_K], c->range_pat[R_P], c->range_pat[R_K], 0, 0};
}

Sched &schedule_key(rtdm_ctx *c, int prod, const std::tuple<int, int, int, int, int> &key);

Sched &schedule(rtdm_ctx *c, int prod) { return schedule_key(c, prod, prod_key(c, prod)); }

// The schedule (triple lists and row runs) of the product with operand and
// output patterns `key`; prod names the kind (run lengths, timing).
Sched &schedule_key(rtdm_ctx *c, int prod, const std::tuple<int, int, int, int, int> &key)
{
    // Row runs: b = 13 products of the column-major path (X H, A tau and the
    // inverse's S X real, U K and W U^dagger complex), b = 4 products with op(A) = A.
    const bool cm_kind = prod == RTDM_PROD_XH || prod == RTDM_PROD_AT || prod == RTDM_PROD_UK ||
                         prod == RTDM_PROD_WU || prod == RTDM_PROD_SX;
    const int nj = std::get<3>(key) != 0 ? 1
                   : c->b == 13 ? (!cm_kind ? 1
                                   : (prod == RTDM_PROD_UK || prod == RTDM_PROD_WU) ? c->run_cplx
                                                                                      : c->run_real)
                   : c->b == 4 ? c->run_b4
                               : 1;
    auto runs_for = [&](Sched &S) {
        // (every kind is scheduled when the ranges are set, so this never runs during a capture)
        if (nj > 1)
            build_runs(S, *c->pats[std::get<0>(key)], *c->pats[std::get<1>(key)], *c->pats[std::get<2>(key)],
                       std::get<4>(key), nj, c->b == 4, c->row_tile);
    };
    auto it = c->scheds.find(key);
    if (it != c->scheds.end()) {
        runs_for(*it->second);   // a kind sharing its patterns with an earlier one (equal cut-offs)
        return *it->second;
    }
    auto S = std::make_unique<Sched>();
    const Pattern &A = *c->pats[std::get<0>(key)];
    const Pattern &B = *c->pats[std::get<1>(key)];
    const Pattern &C = *c->pats[std::get<2>(key)];
    S->nout = C.nnzb;
    DBuf<int64_t> cnt;
    cnt.alloc(S->nout);
    launch_sym_count(nullptr, S->nout, C.d_rowof.p, C.d_col.p, A.d_rowptr.p, A.d_col.p,
                     B.d_rowptr.p, B.d_col.p, cnt.p);
    std::vector<int64_t> h(S->nout + 1, 0);
    RT_HIP(hipMemcpy(h.data() + 1, cnt.p, cnt.bytes(), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < S->nout; ++i) h[i + 1] += h[i];
    S->ntrip = h[S->nout];
    S->off.alloc(S->nout + 1);
    RT_HIP(hipMemcpy(S->off.p, h.data(), S->off.bytes(), hipMemcpyHostToDevice));
    S->trip.alloc(std::max<int64_t>(S->ntrip, 1));
    launch_sym_fill(nullptr, S->nout, C.d_rowof.p, C.d_col.p, A.d_rowptr.p, A.d_col.p, A.d_trans.p,
                    B.d_rowptr.p, B.d_col.p, B.d_trans.p, std::get<3>(key), std::get<4>(key),
                    S->off.p, S->trip.p);
    {
        const std::vector<int32_t> ord = tile_order(C, c->row_tile, 1 << 30);
        S->order.alloc(std::max<size_t>(ord.size(), 1));
        if (!ord.empty())
            RT_HIP(hipMemcpy(S->order.p, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    runs_for(*S);
    RT_HIP(hipDeviceSynchronize());
    Sched &ref = *S;
    c->scheds.emplace(key, std::move(S));
    return ref;
}

hipEvent_t event_at(rtdm_ctx *c, size_t k)
{
    while (c->events.size() <= k) {
        hipEvent_t e;
        RT_HIP(hipEventCreate(&e));
        c->events.push_back(e);
    }
    return c->events[k];
}


void product_key(rtdm_ctx *c, int prod, const std::tuple<int, int, int, int, int> &key, const Mat &A,
                 const Mat &B, Mat &C, double alr, double ali, hipStream_t s);

// C = P_C(alpha op(A) op(B)) with the schedule of `prod`.
void product(rtdm_ctx *c, int prod, const Mat &A, const Mat &B, Mat &C, double alr, double ali,
             hipStream_t s)
{
    product_key(c, prod, prod_key(c, prod), A, B, C, alr, ali, s);
}

// The same with the schedule of operand and output patterns `key` (timed as `prod`).
void product_key(rtdm_ctx *c, int prod, const std::tuple<int, int, int, int, int> &key, const Mat &A,
                 const Mat &B, Mat &C, double alr, double ali, hipStream_t s)
{
    Sched &S = schedule_key(c, prod, key);
    RT_CHECK(A.pat == std::get<0>(key) && B.pat == std::get<1>(key) && C.pat == std::get<2>(key),
             RTDM_E_ARG, std::string("operand patterns do not match product ") + kProdName[prod]);
    SpgemmArgs a;
    a.nout = S.nout;
    a.off = S.off.p;
    a.trip = S.trip.p;
    a.ar = A.re.p;
    a.ai = A.cplx ? A.im.p : nullptr;
    a.br = B.re.p;
    a.bi = B.cplx ? B.im.p : nullptr;
    a.cr = C.re.p;
    a.ci = C.cplx ? C.im.p : nullptr;
    a.b = c->b;
    a.op_a = std::get<3>(key);
    a.op_b = std::get<4>(key);
    a.alpha_re = alr;
    a.alpha_im = ali;
    a.precision = c->prec;
    RT_CHECK(C.cplx || (!A.cplx && !B.cplx && ali == 0.0), RTDM_E_UNSUPPORTED,
             "complex product into a real matrix");
    a.wpb = c->wpb;
    if (c->prec == RTDM_PREC_FP16X2) {
        // per-operand max |x| (both planes) for the power-of-two scales
        const Mat *ops[2] = {&A, &B};
        for (int k = 0; k < 2; ++k) {
            const int64_t ne = elems(c, *ops[k]);
            launch_red_max(s, ne, ops[k]->re.p, c->partials.p);
            launch_red_finish(s, c->partials.p, c->f16_max.p + 8 * k);
            if (ops[k]->cplx) {
                launch_red_max(s, ne, ops[k]->im.p, c->partials.p);
                launch_red_finish(s, c->partials.p, c->f16_max.p + 8 * k + 4);
            } else {
                launch_fill(s, 4, 0.0, c->f16_max.p + 8 * k + 4);
            }
        }
        a.maxabs = c->f16_max.p;
    }
    const bool b4_runs_prec = c->prec == RTDM_PREC_FP64 || c->prec == RTDM_PREC_FP32 ||
                              c->prec == RTDM_PREC_BF16X3 || c->prec == RTDM_PREC_FP16X2;
    if (c->b == 4 && b4_runs_prec && a.op_a == 0 && c->run_b4 > 1) {
        auto r = S.runs.find(c->run_b4);
        if (r != S.runs.end() && r->second->nch > 0) {
            const Runs &R = *r->second;
            a.nj = R.nj;
            a.nch = R.nch;
            a.ch_off = R.off.p;
            a.ch_a = R.a.p;
            a.ch_b = R.b.p;
            a.ch_out = R.out.p;
        }
    }
    auto go = [&]() {
        launch_spgemm(s, a);
    };
    if (c->timing && !c->capturing) {
        const size_t k = 2 * c->recs.size();
        RT_HIP(hipEventRecord(event_at(c, k), s));
        go();
        RT_HIP(hipEventRecord(event_at(c, k + 1), s));
        const double b3 = (double)c->b * c->b * c->b;
        const double sub = (A.cplx ? 2.0 : 1.0) * (B.cplx ? 2.0 : 1.0);
        c->recs.push_back({prod, (int)k, (double)S.ntrip * 2.0 * b3 * sub});
    } else {
        go();
    }
}

bool is_split(int prec) { return prec == RTDM_PREC_BF16X3 || prec == RTDM_PREC_FP16X2; }

// Step product with the column-major copy Acm of the left operand (see
// launch_spgemm_cm); same schedule, timing and flop accounting as product().
void product_cm(rtdm_ctx *c, int prod, const Mat &Acm, const Mat &B, Mat &C, int conj_b, int out_cm,
                double alr, hipStream_t s)
{
    Sched &S = schedule(c, prod);
    auto key = prod_key(c, prod);
    RT_CHECK(Acm.pat == std::get<0>(key) && B.pat == std::get<1>(key) && C.pat == std::get<2>(key),
             RTDM_E_ARG, std::string("operand patterns do not match product ") + kProdName[prod]);
    SpgemmArgs a;
    a.nout = S.nout;
    a.off = S.off.p;
    a.trip = S.trip.p;
    a.ar = Acm.re.p;
    a.ai = Acm.cplx ? Acm.im.p : nullptr;
    a.br = B.re.p;
    a.bi = B.cplx ? B.im.p : nullptr;
    a.cr = C.re.p;
    a.ci = C.cplx ? C.im.p : nullptr;
    a.b = c->b;
    a.alpha_re = alr;
    a.zero = c->zero.p;
    a.order = S.order.p;
    a.wpb = c->wpb;
    a.precision = c->prec;
    {
        // row runs of the length chosen for real or complex operands, if built
        const int nj = (!Acm.cplx && !B.cplx) ? c->run_real : c->run_cplx;
        auto r = S.runs.find(nj);
        if (nj > 1 && r != S.runs.end() && r->second->nch > 0) {
            const Runs &R = *r->second;
            a.nj = R.nj;
            a.nch = R.nch;
            a.ch_off = R.off.p;
            a.ch_a = R.a.p;
            a.ch_b = R.b.p;
            a.ch_out = R.out.p;
            a.ch_order = R.order.p;
            a.ch_seg = R.seg.p;
        }
    }
    RT_CHECK(C.cplx || (!Acm.cplx && !B.cplx), RTDM_E_UNSUPPORTED, "complex product into a real matrix");
    const bool split = is_split(c->prec);
    if (c->prec == RTDM_PREC_FP16X2) {
        // max |x| of both (real) operands for the power-of-two scales
        const Mat *ops[2] = {&Acm, &B};
        for (int k = 0; k < 2; ++k) {
            launch_red_max(s, elems(c, *ops[k]), ops[k]->re.p, c->partials.p);
            launch_red_finish(s, c->partials.p, c->f16_max.p + 8 * k);
            launch_fill(s, 4, 0.0, c->f16_max.p + 8 * k + 4);
        }
        a.maxabs = c->f16_max.p;
    }
    auto go = [&]() {
        if (split) launch_spgemm_cm_split(s, a);
        else launch_spgemm_cm(s, a, conj_b, out_cm);
    };
    if (c->timing && !c->capturing) {
        const size_t k = 2 * c->recs.size();
        RT_HIP(hipEventRecord(event_at(c, k), s));
        go();
        RT_HIP(hipEventRecord(event_at(c, k + 1), s));
        const double b3 = (double)c->b * c->b * c->b;
        const double sub = (Acm.cplx ? 2.0 : 1.0) * (B.cplx ? 2.0 : 1.0);
        c->recs.push_back({prod, (int)k, (double)S.ntrip * 2.0 * b3 * sub});
    } else {
        go();
    }
}

// Column-major copy of every block of M (both planes).
void transpose_into(rtdm_ctx *c, const Mat &M, Mat &out, hipStream_t s)
{
    const int64_t nb = c->pats[M.pat]->nnzb;
    launch_transpose_blocks(s, nb, c->b, M.re.p, out.re.p);
    if (M.cplx) launch_transpose_blocks(s, nb, c->b, M.im.p, out.im.p);
}

bool use_cm(rtdm_ctx *c) { return c->b == 13 && (c->prec == RTDM_PREC_FP64 || c->prec == RTDM_PREC_FP32); }

void reduce_finish(rtdm_ctx *c, hipStream_t s, double *out) { launch_red_finish(s, c->partials.p, out); }

void read_scalars(double *dst, const double *src, int n, hipStream_t s)
{
    RT_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
}

void ensure_charges(rtdm_ctx *c, hipStream_t s)
{
    if (c->charges_valid) return;
    Pattern &ps = pat_of(c, R_HS);
    for (int k = 0; k < n_kicks(c); ++k)
        launch_mulliken(s, c->n, c->b, ps.d_rowptr.p, ps.d_trans.p, c->s_to_k.p, c->mats[RTDM_MAT_S].re.p,
                        kmat(c, k).re.p, qcur(c, k));
    RT_HIP(hipMemcpyAsync(c->q_prev, c->q_cur, n_kicks(c) * c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (!c->q_ref_valid) {
        RT_HIP(hipMemcpyAsync(c->q_ref.p, c->q_cur, c->n * sizeof(double), hipMemcpyDeviceToDevice, s));
        c->q_ref_valid = true;
    }
    c->charges_valid = true;
}

void ensure_s_norm(rtdm_ctx *c, hipStream_t s)
{
    if (c->s_norm_valid) return;
    launch_red_sumsq(s, elems(c, c->mats[RTDM_MAT_S]), c->mats[RTDM_MAT_S].re.p, c->partials.p);
    reduce_finish(c, s, c->s_norm2.p);
    if (c->mixed) launch_add_scalar(s, c->s_norm2.p, -(double)c->n_pad);   // the padded identity's ones
    c->s_norm_valid = true;
}

// Arithmetic of the step's products under the options' precision: the forms
// that reduce every product, else FP64 (the *_TAYLOR forms lower only late
// Taylor terms, inside build_propagator).
int all_products_prec(rtdm_ctx *c)
{
    switch (c->opt.precision) {
    case RTDM_PREC_FP32:
    case RTDM_PREC_BF16X3:
    case RTDM_PREC_FP16X2: return c->opt.precision;
    default: return RTDM_PREC_FP64;
    }
}

// U = sum_{n=0}^{p} (-i)^n tau_n with tau_0 = I, tau_1 = dt A, tau_n = (dt/n) P_P(A tau_{n-1}).
void build_propagator(rtdm_ctx *c, double dt, hipStream_t s)
{
    Mat &A = c->mats[RTDM_MAT_A];
    Mat &U = c->mats[RTDM_MAT_U];
    const int64_t ne = elems(c, A);
    const int p = c->opt.taylor_order;
    const bool low32 = c->opt.precision == RTDM_PREC_FP32_TAYLOR && c->Ac32.p != nullptr;
    // BF16x3 late terms at b = 4 over row runs: operands stored split (the
    // FP32 buffers hold the hi and lo planes), the sum into U fused
    const bool low16 = c->opt.precision == RTDM_PREC_BF16X3_TAYLOR && c->b == 4 && c->Ac32.p != nullptr &&
                       c->run_b4 == 16 && [&] {
                           Sched &S = schedule(c, RTDM_PROD_AT);
                           auto r = S.runs.find(16);
                           return r != S.runs.end() && r->second->nch > 0;
                       }();
    auto as16 = [](float *p) { return reinterpret_cast<short *>(p); };
    int n0 = 2, low = all_products_prec(c);
    switch (c->opt.precision) {
    case RTDM_PREC_FP64: n0 = p + 1; break;
    case RTDM_PREC_FP32_TAYLOR: n0 = c->opt.taylor_low_from; low = RTDM_PREC_FP32; break;
    case RTDM_PREC_BF16X3_TAYLOR: n0 = c->opt.taylor_low_from; low = RTDM_PREC_BF16X3; break;
    case RTDM_PREC_FP16X2_TAYLOR: n0 = c->opt.taylor_low_from; low = RTDM_PREC_FP16X2; break;
    default: break;
    }
    launch_fill(s, ne, 0.0, U.re.p);   // kernels, not memsets: this code may be captured in a graph
    launch_fill(s, ne, 0.0, U.im.p);
    launch_add_identity(s, c->n, c->b, pat_of(c, R_P).d_diag.p, 1.0, U.re.p);
    if (p >= 1) {
        launch_axpby(s, ne, dt, A.re.p, 0.0, nullptr, c->tau[0].re.p);
        launch_axpby(s, ne, -1.0, c->tau[0].re.p, 1.0, U.im.p, U.im.p);
    }
    // (-i)^k: k%4 == 0 -> +Re, 1 -> -Im, 2 -> -Re, 3 -> +Im
    auto add_term = [&](int k, const double *t64, const float *t32) {
        const double sign = (k % 4 == 0 || k % 4 == 3) ? 1.0 : -1.0;
        double *dst = (k % 2 == 0) ? U.re.p : U.im.p;
        if (t64) launch_axpby(s, ne, sign, t64, 1.0, dst, dst);
        else launch_axpy_f32(s, ne, sign, t32, dst);
    };
    int cur = 0;          // tau[cur] (FP64) or tau32[cur] (FP32 or split BF16) holds tau_{k-1}
    bool in32 = false;
    if (low16 && n0 <= p) launch_to_bf16x2(s, pat_of(c, R_P).nnzb, 0, A.re.p, as16(c->Ac32.p));
    // FP32 copy of A: of its column-major copy at b = 13, of A itself (row-major) at b = 4
    if (low32 && n0 <= p)
        launch_to_f32(s, pat_of(c, R_P).nnzb, c->b, 0, c->b == 13 ? c->Ac.re.p : A.re.p, c->Ac32.p);
    for (int k = 2; k <= p; ++k) {
        if (low16 && k >= n0) {
            if (!in32) {
                launch_to_bf16x2(s, pat_of(c, R_P).nnzb, 1, c->tau[cur].re.p, as16(c->tau32[cur].p));
                in32 = true;
            }
            Sched &S = schedule(c, RTDM_PROD_AT);
            const Runs &R = *S.runs.find(16)->second;
            SpgemmArgs a;
            a.nout = S.nout;
            a.b = c->b;
            a.alpha_re = dt / k;
            a.nj = R.nj;
            a.nch = R.nch;
            a.ch_off = R.off.p;
            a.ch_a = R.a.p;
            a.ch_b = R.b.p;
            a.ch_out = R.out.p;
            // (-i)^k: k%4 == 0 -> +Re, 1 -> -Im, 2 -> -Re, 3 -> +Im
            const double sign = (k % 4 == 0 || k % 4 == 3) ? 1.0 : -1.0;
            double *udst = (k % 2 == 0) ? U.re.p : U.im.p;
            const bool more = k < p;
            const bool rec = c->timing && !c->capturing;
            const size_t ev = 2 * c->recs.size();
            if (rec) RT_HIP(hipEventRecord(event_at(c, ev), s));
            launch_spgemm_r16(s, a, as16(c->Ac32.p), as16(c->tau32[cur].p), more ? as16(c->tau32[1 - cur].p) : nullptr,
                              udst, sign);
            if (rec) {
                RT_HIP(hipEventRecord(event_at(c, ev + 1), s));
                const double b3 = (double)c->b * c->b * c->b;
                c->recs.push_back({RTDM_PROD_AT, (int)ev, (double)S.ntrip * 2.0 * b3});
            }
        } else if (low32 && k >= n0) {
            if (!in32) {
                launch_to_f32(s, pat_of(c, R_P).nnzb, c->b, 0, c->tau[cur].re.p, c->tau32[cur].p);
                in32 = true;
            }
            Sched &S = schedule(c, RTDM_PROD_AT);
            SpgemmArgs a;
            a.nout = S.nout;
            a.off = S.off.p;
            a.trip = S.trip.p;
            a.b = c->b;
            a.alpha_re = dt / k;
            a.order = S.order.p;
            a.wpb = c->wpb;
            const int nj = c->b == 4 ? c->run_b4 : c->run_real;
            if (nj > 1) {
                auto rr = S.runs.find(nj);
                if (rr != S.runs.end() && rr->second->nch > 0) {
                    const Runs &R = *rr->second;
                    a.nj = R.nj;
                    a.nch = R.nch;
                    a.ch_off = R.off.p;
                    a.ch_a = R.a.p;
                    a.ch_b = R.b.p;
                    a.ch_out = R.out.p;
                    a.ch_order = R.order.p;
                    a.ch_seg = R.seg.p;
                }
            }
            const bool rec = c->timing && !c->capturing;
            const size_t ev = 2 * c->recs.size();
            if (rec) RT_HIP(hipEventRecord(event_at(c, ev), s));
            launch_spgemm_r32(s, a, c->Ac32.p, c->tau32[cur].p, c->tau32[1 - cur].p, c->zero32.p);
            if (rec) {
                RT_HIP(hipEventRecord(event_at(c, ev + 1), s));
                const double b3 = (double)c->b * c->b * c->b;
                c->recs.push_back({RTDM_PROD_AT, (int)ev, (double)S.ntrip * 2.0 * b3});
            }
            add_term(k, nullptr, c->tau32[1 - cur].p);
        } else {
            Mat &src = c->tau[cur];
            Mat &dst = c->tau[1 - cur];
            const int saved = c->prec;
            if (k >= n0) c->prec = low;
            // the *_TAYLOR split forms keep the step in FP64, so the column-major A is current
            const bool split_cm = c->b == 13 && is_split(c->prec) &&
                                  (c->opt.precision == RTDM_PREC_BF16X3_TAYLOR ||
                                   c->opt.precision == RTDM_PREC_FP16X2_TAYLOR);
            if (use_cm(c) || split_cm) product_cm(c, RTDM_PROD_AT, c->Ac, src, dst, 0, 0, dt / k, s);
            else product(c, RTDM_PROD_AT, A, src, dst, dt / k, 0.0, s);
            c->prec = saved;
            add_term(k, dst.re.p, nullptr);
        }
        cur = 1 - cur;
    }
    if (use_cm(c)) transpose_into(c, U, c->Uc, s);
}

// D = P_P(U^dagger P_P(S U)) - S; sums into c->unit_sums.
void unitarity_sums(rtdm_ctx *c, hipStream_t s)
{
    Mat &U = c->mats[RTDM_MAT_U];
    product(c, RTDM_PROD_SX, c->mats[RTDM_MAT_S], U, c->V, 1.0, 0.0, s);
    product(c, RTDM_PROD_UV, U, c->V, c->Z, 1.0, 0.0, s);
    launch_red_unitarity(s, pat_of(c, R_P).nnzb, c->b, c->p_to_hs.p, c->mats[RTDM_MAT_S].re.p,
                         c->Z.re.p, c->Z.im.p, c->partials.p);
    reduce_finish(c, s, c->unit_sums.p);
    ensure_s_norm(c, s);
}

void drop_graph(rtdm_ctx *c)
{
    c->graph_epoch++;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->gexec_multi) (void)hipGraphExecDestroy(c->gexec_multi);
    if (c->graph_multi) (void)hipGraphDestroy(c->graph_multi);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gexec_multi = nullptr;
    c->graph_multi = nullptr;
}

void ensure_obs(rtdm_ctx *c, int64_t rows)
{
    const int64_t G = c->n_groups > 1 ? c->n_groups : 0;
    const int NK = n_kicks(c);
    if (rows <= c->obs_cap && (int64_t)c->obs.n >= c->obs_cap * 8 * NK &&
        (G == 0 || (int64_t)c->obs_g.n >= c->obs_cap * G * 4 * NK))
        return;
    int64_t cap = std::max<int64_t>(2 * c->obs_cap, 1024);
    while (cap < rows) cap *= 2;
    // earlier steps may still write rows on the caller's stream: let them land
    RT_HIP(hipDeviceSynchronize());
    // one trace of cap rows per kick, each kick's rows contiguous
    DBuf<double> nb;
    nb.alloc(cap * 8 * NK);
    if (c->obs_rows > 0 && c->obs.p)
        for (int k = 0; k < NK; ++k)
            RT_HIP(hipMemcpy(nb.p + k * cap * 8, obs_of(c, k), c->obs_rows * 8 * sizeof(double),
                             hipMemcpyDeviceToDevice));
    if (G > 0) {
        DBuf<double> ng;
        ng.alloc(cap * G * 4 * NK);
        if (c->obs_rows > 0 && c->obs_g.p)
            for (int k = 0; k < NK; ++k)
                RT_HIP(hipMemcpy(ng.p + k * cap * G * 4, obs_g_of(c, k), c->obs_rows * G * 4 * sizeof(double),
                                 hipMemcpyDeviceToDevice));
        c->obs_g = std::move(ng);
    }
    c->obs = std::move(nb);
    c->obs_cap = cap;
    drop_graph(c);   // the captured step refers to the trace buffers
}

void require(bool cond, const char *msg) { RT_CHECK(cond, RTDM_E_STATE, msg); }

void upload_planes(rtdm_ctx *c, int m, const double *re, const double *im, hipStream_t s)
{
    Mat &M = c->mats[m];
    const int64_t ne = elems(c, M);
    RT_HIP(hipMemcpyAsync(M.re.p, re, ne * sizeof(double), hipMemcpyHostToDevice, s));
    if (M.cplx) {
        if (im) RT_HIP(hipMemcpyAsync(M.im.p, im, ne * sizeof(double), hipMemcpyHostToDevice, s));
        else RT_HIP(hipMemsetAsync(M.im.p, 0, M.im.bytes(), s));
    }
    RT_HIP(hipStreamSynchronize(s));
}

void after_upload(rtdm_ctx *c, int m)
{
    c->uploaded[m] = true;
    switch (m) {
    case RTDM_MAT_S:
        c->X_valid = false;
        c->U_valid = false;
        c->A0_valid = false;
        c->s_norm_valid = false;
        c->charges_valid = false;
        c->q_ref_valid = false;
        break;
    case RTDM_MAT_H0: c->U_valid = false; c->A0_valid = false; break;
    case RTDM_MAT_X: c->X_valid = true; c->U_valid = false; c->Xc_valid = false; c->A0_valid = false; break;
    case RTDM_MAT_K:
        for (int k = 1; k < n_kicks(c); ++k) {   // every kick starts from the uploaded K
            const int64_t ne = elems(c, c->mats[RTDM_MAT_K]);
            RT_HIP(hipMemcpy(c->Kx[k - 1].re.p, c->mats[RTDM_MAT_K].re.p, ne * sizeof(double),
                             hipMemcpyDeviceToDevice));
            RT_HIP(hipMemcpy(c->Kx[k - 1].im.p, c->mats[RTDM_MAT_K].im.p, ne * sizeof(double),
                             hipMemcpyDeviceToDevice));
        }
        c->charges_valid = false;
        c->q_ref_valid = false;
        c->obs_reset_pending = true;
        c->obs_rows = 0;
        c->t_now = 0.0;
        c->step_count = 0;
        c->trace_dt_mixed = false;
        c->herm_valid = false;
        break;
    case RTDM_MAT_U: c->U_valid = true; c->u_copies_valid = false; break;
    case RTDM_MAT_W: c->W_in_cm = false; break;
    default: break;
    }
}

void mlp_configure(rtdm_ctx *c)
{
    MlpState &M = c->mlp;
    RT_CHECK(c->b > 0, RTDM_E_STATE, "set_geometry first");
    if (M.b == c->b && M.np > 0) return;
    M = MlpState();
    M.b = c->b;
    M.in = 4 + c->b * c->b;
    M.out = c->b * c->b;
    M.nw1 = (int64_t)kMlpHidden * M.in;
    M.nb1 = kMlpHidden;
    M.nw2 = (int64_t)M.out * kMlpHidden;
    M.nb2 = M.out;
    M.np = M.nw1 + M.nb1 + M.nw2 + M.nb2;
    M.w.alloc(M.np);
    M.m.alloc(M.np);
    M.v.alloc(M.np);
    M.grad.alloc(M.np);
    M.w1h.alloc(M.nw1);
    M.w2h.alloc(M.nw2);
    M.dsum.alloc(1);
}

void mlp_sync_half(rtdm_ctx *c, hipStream_t s)
{
    MlpState &M = c->mlp;
    launch_to_half(s, M.nw1, M.w.p, M.w1h.p);
    launch_to_half(s, M.nw2, M.w.p + M.nw1 + M.nb1, M.w2h.p);
}

void mlp_work(rtdm_ctx *c, int64_t n)
{
    MlpState &M = c->mlp;
    if (n <= M.work_n) return;
    M.hid.alloc((size_t)n * kMlpHidden);
    M.y.alloc((size_t)n * M.out);
    M.dy.alloc((size_t)n * M.out);
    M.dh.alloc((size_t)n * kMlpHidden);
    M.sqerr.alloc(n);
    M.work_n = n;
}

const float *mlp_b1(const MlpState &M) { return M.w.p + M.nw1; }
const float *mlp_b2(const MlpState &M) { return M.w.p + M.nw1 + M.nb1 + M.nw2; }

// loss (mean squared error per output element) and gradient of n samples
// (x_idx selects rows of x and t; null = rows 0..n-1).
double mlp_loss_grad(rtdm_ctx *c, int64_t n, const int32_t *idx, const float *x, const float *t, hipStream_t s)
{
    MlpState &M = c->mlp;
    mlp_work(c, n);
    launch_mlp_forward(s, n, M.in, M.out, idx, x, M.w1h.p, mlp_b1(M), M.w2h.p, mlp_b2(M), M.hid.p, M.y.p);
    launch_mlp_delta(s, n, M.out, idx, t, M.y.p, M.hid.p, M.w2h.p, M.dy.p, M.dh.p, M.sqerr.p);
    launch_mlp_grad(s, n, M.in, M.out, idx, x, M.hid.p, M.dy.p, M.dh.p, M.grad.p);
    launch_sum_f32(s, n, M.sqerr.p, M.dsum.p);
    double sum = 0.0;
    read_scalars(&sum, M.dsum.p, 1, s);
    return sum / ((double)n * M.out);
}

}  // namespace

// ================================================================== ABI

#define API_BEGIN DevMemScope devmem_scope_((c) ? &(c)->mem : nullptr); try {
#define API_END(c)                                                \
    }                                                             \
    catch (const rtdm::Error &e) {                                \
        if (c) (c)->err = e.what();                               \
        return e.code;                                            \
    }                                                             \
    catch (const std::bad_alloc &) {                              \
        if (c) (c)->err = "host allocation failed";               \
        return RTDM_E_OOM;                                        \
    }                                                             \
    catch (const std::exception &e) {                             \
        if (c) (c)->err = e.what();                               \
        return RTDM_E_ARG;                                        \
    }                                                             \
    if (c) (c)->err.clear();                                      \
    return RTDM_OK;

extern "C" {

int rtdm_default_options(rtdm_options *opt)
{
    if (!opt) return RTDM_E_ARG;
    opt->taylor_order = 5;
    opt->unit_check_every = 0;
    opt->precision = RTDM_PREC_FP64;
    opt->h_model = RTDM_HMODEL_FIXED;
    opt->h_gain = 0.5;
    opt->inv_start = RTDM_INV_BLOCK_JACOBI;
    opt->inv_tol = 1e-10;
    opt->inv_max_iter = 50;
    opt->taylor_low_from = 3;
    opt->use_graph = 0;
    opt->propagator = RTDM_PROP_EM;
    opt->sc_steps = 0;
    opt->sc_iters = 2;
    opt->unit_tol = 0.0;
    opt->graph_steps = 16;
    opt->n_kicks = 1;
    opt->xh_every_step = 0;
    return RTDM_OK;
}

int rtdm_create(rtdm_ctx **out, int hip_device, const rtdm_options *opt)
{
    if (!out) return RTDM_E_ARG;
    *out = nullptr;
    rtdm_ctx *c = nullptr;
    try {
        c = new rtdm_ctx();
    } catch (...) {
        return RTDM_E_OOM;
    }
    API_BEGIN
    int ndev = 0;
    RT_HIP(hipGetDeviceCount(&ndev));
    RT_CHECK(hip_device >= 0 && hip_device < ndev, RTDM_E_ARG, "no such HIP device");
    c->device = hip_device;
    if (opt) c->opt = *opt;
    else rtdm_default_options(&c->opt);
    RT_CHECK(c->opt.taylor_order >= 0 && c->opt.taylor_order <= 32, RTDM_E_ARG, "taylor_order out of range");
    RT_CHECK(c->opt.precision >= RTDM_PREC_FP64 && c->opt.precision <= RTDM_PREC_FP16X2_TAYLOR, RTDM_E_ARG,
             "unknown precision");
    RT_CHECK(c->opt.h_model == RTDM_HMODEL_FIXED || c->opt.h_model == RTDM_HMODEL_MULLIKEN, RTDM_E_ARG,
             "unknown h_model");
    RT_CHECK(c->opt.inv_start >= 0 && c->opt.inv_start <= RTDM_INV_LEARNED, RTDM_E_ARG, "unknown inv_start");
    RT_CHECK(c->opt.inv_max_iter >= 1 && c->opt.inv_tol > 0, RTDM_E_ARG, "bad inverse options");
    RT_CHECK(c->opt.unit_check_every >= 0, RTDM_E_ARG, "unit_check_every < 0");
    RT_CHECK(c->opt.taylor_low_from >= 2, RTDM_E_ARG, "taylor_low_from < 2");
    RT_CHECK(c->opt.propagator >= RTDM_PROP_EM && c->opt.propagator <= RTDM_PROP_M4, RTDM_E_ARG,
             "unknown propagator");
    RT_CHECK(c->opt.propagator == RTDM_PROP_EM || c->opt.precision == RTDM_PREC_FP64, RTDM_E_UNSUPPORTED,
             "ETRS and M4 need RTDM_PREC_FP64");
    RT_CHECK(c->opt.sc_steps >= 0 && c->opt.sc_iters >= 0, RTDM_E_ARG, "sc_steps / sc_iters < 0");
    RT_CHECK(c->opt.unit_tol >= 0.0, RTDM_E_ARG, "unit_tol < 0");
    RT_CHECK(c->opt.graph_steps >= 1 && c->opt.graph_steps <= 1024, RTDM_E_ARG, "graph_steps outside 1..1024");
    RT_CHECK(c->opt.n_kicks >= 1 && c->opt.n_kicks <= 8, RTDM_E_ARG, "n_kicks outside 1..8");
    RT_CHECK(c->opt.xh_every_step == 0 || c->opt.xh_every_step == 1, RTDM_E_ARG, "xh_every_step must be 0 or 1");
    RT_CHECK(c->opt.n_kicks == 1 || (c->opt.h_model == RTDM_HMODEL_FIXED && c->opt.sc_steps == 0),
             RTDM_E_UNSUPPORTED, "several kicks share one propagator: they need a fixed H and no corrector");
    set_device(c);
    (void)static_scratch(c->device);   // device address of rtdm_multiply_noalloc's scratch on this GPU
    if (const char *e = getenv("RTDM_RUN_REAL")) c->run_real = atoi(e);
    if (const char *e = getenv("RTDM_RUN_CPLX")) c->run_cplx = atoi(e);
    if (const char *e = getenv("RTDM_ROW_TILE")) c->row_tile = std::max(1, atoi(e));
    if (const char *e = getenv("RTDM_RUN_B4")) c->run_b4 = atoi(e);
    RT_CHECK(c->run_b4 == 1 || c->run_b4 == 16, RTDM_E_ARG, "b = 4 row runs hold 1 or 16 outputs");
    RT_CHECK((c->run_real >= 1 && c->run_real <= 4) || c->run_real == 8, RTDM_E_ARG,
             "row runs of 1 to 4 or 8 outputs for real products");
    RT_CHECK(c->run_cplx >= 1 && c->run_cplx <= 4, RTDM_E_ARG,
             "row runs of 1 to 4 outputs for complex products");
    c->partials.alloc(kRedBlocks * 4);
    c->herm_sums.alloc(4 * c->opt.n_kicks);
    c->unit_sums.alloc(4);
    c->s_norm2.alloc(4);
    c->hot_sums.alloc(4);
    c->obs_tmp.alloc(8);
    c->f16_max.alloc(16);
    c->zero.alloc(256);
    RT_HIP(hipMemset(c->zero.p, 0, c->zero.bytes()));
    *out = c;
    }
    catch (const rtdm::Error &e) {
        const int code = e.code;
        delete c;
        return code;
    }
    catch (...) {
        delete c;
        return RTDM_E_HIP;
    }
    return RTDM_OK;
}

int rtdm_destroy(rtdm_ctx *c)
{
    if (!c) return RTDM_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto e : c->events) (void)hipEventDestroy(e);
    drop_graph(c);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    delete c;
    return RTDM_OK;
}

int rtdm_set_geometry(rtdm_ctx *c, int64_t n_atoms, const double *xyz, const int32_t *nbf)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(n_atoms >= 1 && n_atoms < (int64_t)INT32_MAX && xyz && nbf, RTDM_E_ARG, "bad geometry arguments");
    RT_CHECK(!c->mem.base, RTDM_E_STATE, "the geometry is fixed once a workspace is bound");
    int b = 0;
    bool mixed = false;
    for (int64_t i = 0; i < n_atoms; ++i) {
        RT_CHECK(nbf[i] >= 1 && nbf[i] <= 16, RTDM_E_UNSUPPORTED, "functions per atom must be 1..16");
        b = std::max(b, (int)nbf[i]);
        mixed |= nbf[i] != nbf[0];
    }
    if (mixed) {
        RT_CHECK(b == 4 || b == 13, RTDM_E_UNSUPPORTED,
                 "mixed block sizes need a largest size of 4 or 13 (the padded size)");
        RT_CHECK(c->opt.precision == RTDM_PREC_FP64 && c->opt.inv_start != RTDM_INV_COLD &&
                     c->opt.inv_start != RTDM_INV_LEARNED,
                 RTDM_E_UNSUPPORTED, "mixed block sizes run FP64 products with the block-Jacobi or previous start");
    }
    for (int64_t e = 0; e < 3 * n_atoms; ++e) RT_CHECK(std::isfinite(xyz[e]), RTDM_E_ARG, "non-finite position");
    RT_HIP(hipDeviceSynchronize());
    c->scheds.clear();
    c->pats.clear();
    for (auto &m : c->mats) { m.re.release(); m.im.release(); m.pat = -1; }
    c->ranges_set = false;
    c->n = n_atoms;
    c->b = b;
    c->mixed = mixed;
    c->nbf.assign(nbf, nbf + n_atoms);
    c->n_pad = 0;
    for (int64_t i = 0; i < n_atoms; ++i) c->n_pad += b - nbf[i];
    if (mixed) {
        c->d_nbf.alloc(n_atoms);
        RT_HIP(hipMemcpy(c->d_nbf.p, nbf, c->d_nbf.bytes(), hipMemcpyHostToDevice));
    } else {
        c->d_nbf.release();
    }
    c->xyz.assign(xyz, xyz + 3 * n_atoms);
    c->d_xyz.alloc(3 * n_atoms);
    RT_HIP(hipMemcpy(c->d_xyz.p, xyz, c->d_xyz.bytes(), hipMemcpyHostToDevice));
    std::fill(std::begin(c->uploaded), std::end(c->uploaded), false);
    c->X_valid = c->U_valid = c->charges_valid = c->q_ref_valid = c->s_norm_valid = false;
    API_END(c)
}

int rtdm_set_ranges(rtdm_ctx *c, double R_hs, double R_p, double R_k)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    RT_CHECK(!c->mem.base, RTDM_E_STATE, "the ranges are fixed once a workspace is bound");
    set_device(c);
    require(c->n > 0, "set_geometry first");
    RT_CHECK(std::isfinite(R_hs) && std::isfinite(R_k) && std::isfinite(R_p) && R_hs >= 0 && R_k >= 0,
             RTDM_E_ARG, "bad ranges");
    if (R_p <= 0) R_p = std::max(R_hs, R_k);
    RT_HIP(hipDeviceSynchronize());
    c->scheds.clear();
    c->pats.clear();
    const double r[3] = {R_hs, R_p, R_k};
    for (int a = 0; a < 3; ++a) {
        c->radius[a] = r[a];
        c->range_pat[a] = -1;
        for (int q = 0; q < a; ++q)
            if (r[q] == r[a]) c->range_pat[a] = c->range_pat[q];
        if (c->range_pat[a] < 0) {
            auto P = std::make_unique<Pattern>();
            build_pattern(*P, c->xyz, c->n, r[a]);
            c->pats.push_back(std::move(P));
            c->range_pat[a] = (int)c->pats.size() - 1;
        }
    }
    for (int m = 0; m < RTDM_MAT_COUNT; ++m) alloc_mat(c, c->mats[m], slot_range(m), slot_complex(m));
    alloc_mat(c, c->tau[0], R_P, false);
    alloc_mat(c, c->tau[1], R_P, false);
    if (c->opt.h_model == RTDM_HMODEL_MULLIKEN && !c->opt.xh_every_step) alloc_mat(c, c->A0, R_P, false);
    else c->A0.re.release();
    c->A0_valid = false;
    alloc_mat(c, c->Kn, R_K, true);
    alloc_mat(c, c->Xn, R_P, false);
    alloc_mat(c, c->Wh, R_P, false);
    alloc_mat(c, c->V, R_P, true);
    alloc_mat(c, c->Z, R_P, true);
    c->Ac32.release();
    c->tau32[0].release();
    c->tau32[1].release();
    // FP32 copies of A and tau (FP32 late Taylor terms), or at b = 4 the same
    // bytes as BF16 hi / lo planes (BF16x3 late Taylor terms)
    if (((c->b == 13 || c->b == 4) && c->opt.precision == RTDM_PREC_FP32_TAYLOR) ||
        (c->b == 4 && c->opt.precision == RTDM_PREC_BF16X3_TAYLOR)) {
        const int64_t ne = pat_of(c, R_P).nnzb * (int64_t)c->b * c->b;
        c->Ac32.alloc(ne);
        c->tau32[0].alloc(ne);
        c->tau32[1].alloc(ne);
        c->zero32.alloc(256);
        RT_HIP(hipMemset(c->zero32.p, 0, c->zero32.bytes()));
    }
    if (c->b == 13) {
        alloc_mat(c, c->Xc, R_P, false);
        alloc_mat(c, c->Ac, R_P, false);
        alloc_mat(c, c->Uc, R_P, true);
        alloc_mat(c, c->Wc, R_K, true);
        alloc_mat(c, c->Sc, R_HS, false);
    }
    c->Xc_valid = false;
    c->W_in_cm = false;
    if (c->opt.propagator != RTDM_PROP_EM) {
        alloc_mat(c, c->E1, R_P, true);
        alloc_mat(c, c->E2, R_P, true);
        alloc_mat(c, c->E3, R_P, true);
        alloc_mat(c, c->A1, R_P, false);
    }
    if (c->opt.sc_steps > 0 && c->opt.sc_iters > 0) {
        alloc_mat(c, c->Kt, R_K, true);
        c->q_c.alloc(c->n);
    }
    // maps between patterns
    Pattern &ps = pat_of(c, R_HS), &pk = pat_of(c, R_K), &pp = pat_of(c, R_P);
    auto find = [](const Pattern &P, int64_t i, int32_t j) -> int32_t {
        auto b0 = P.col.begin() + P.rowptr[i], b1 = P.col.begin() + P.rowptr[i + 1];
        auto it = std::lower_bound(b0, b1, j);
        return (it != b1 && *it == j) ? (int32_t)(it - P.col.begin()) : -1;
    };
    std::vector<int32_t> s2k(ps.nnzb), p2s(pp.nnzb);
    for (int64_t p = 0; p < ps.nnzb; ++p) s2k[p] = find(pk, ps.rowof[p], ps.col[p]);
    for (int64_t p = 0; p < pp.nnzb; ++p) p2s[p] = find(ps, pp.rowof[p], pp.col[p]);
    std::vector<int32_t> s2p(ps.nnzb), iota(ps.nnzb);
    for (int64_t p = 0; p < ps.nnzb; ++p) {
        s2p[p] = find(pp, ps.rowof[p], ps.col[p]);
        iota[p] = (int32_t)p;
    }
    c->hs_to_p.alloc(ps.nnzb);
    c->hs_iota.alloc(ps.nnzb);
    RT_HIP(hipMemcpy(c->hs_to_p.p, s2p.data(), c->hs_to_p.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(c->hs_iota.p, iota.data(), c->hs_iota.bytes(), hipMemcpyHostToDevice));
    c->s_to_k.alloc(ps.nnzb);
    c->p_to_hs.alloc(pp.nnzb);
    RT_HIP(hipMemcpy(c->s_to_k.p, s2k.data(), c->s_to_k.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(c->p_to_hs.p, p2s.data(), c->p_to_hs.bytes(), hipMemcpyHostToDevice));
    c->q_ref.alloc(c->n);
    c->q_a.alloc(c->n * n_kicks(c));
    c->q_b.alloc(c->n * n_kicks(c));
    c->q_cur = c->q_a.p;
    c->q_prev = c->q_b.p;
    c->Kx.clear();
    c->Kx.resize(n_kicks(c) - 1);
    for (auto &Km : c->Kx) alloc_mat(c, Km, R_K, true);
    c->kick_sel = 0;
    c->atom_max.alloc(c->n);
    c->scratch.alloc((size_t)c->n * c->b * 2 * c->b);
    drop_graph(c);
    c->n_groups = 1;
    c->gptr.clear();
    c->obs_g.release();
    {
        double cen[3];
        exact_centre(c->xyz, 0, c->n, cen);
        c->d_centre.alloc(3);
        c->d_centre_all.alloc(3);
        RT_HIP(hipMemcpy(c->d_centre.p, cen, sizeof(cen), hipMemcpyHostToDevice));
        RT_HIP(hipMemcpy(c->d_centre_all.p, cen, sizeof(cen), hipMemcpyHostToDevice));
    }
    c->step_count = 0;
    c->trace_dt_mixed = false;
    c->step_st.alloc(2);
    c->step_tt.alloc(2);
    c->obs_reset_pending = true;
    c->obs_cap = 0;
    ensure_obs(c, 1024);
    c->obs_rows = 0;
    c->t_now = 0.0;
    std::fill(std::begin(c->uploaded), std::end(c->uploaded), false);
    c->X_valid = c->U_valid = c->charges_valid = c->q_ref_valid = c->s_norm_valid = false;
    c->herm_valid = false;
    c->ranges_set = true;
    for (int prod : {RTDM_PROD_XH, RTDM_PROD_AT, RTDM_PROD_UK, RTDM_PROD_WU, RTDM_PROD_SX}) schedule(c, prod);
    {
        // W U^dagger over rows of a stored U^dagger where the b = 4 FP64 products run
        // over row runs of 16 (not the split form of small systems)
        Sched &uk = schedule(c, RTDM_PROD_UK);
        auto r = uk.runs.find(16);
        c->Uh_on = c->b == 4 && c->run_b4 == 16 && all_products_prec(c) == RTDM_PREC_FP64 && r != uk.runs.end() &&
                   r->second->nch > 0 && !b4_split_form(r->second->nch);
        if (c->Uh_on) {
            alloc_mat(c, c->Uh, R_P, true);
            schedule_key(c, RTDM_PROD_WU, wuh_key(c));
        } else {
            c->Uh.re.release();
            c->Uh.im.release();
        }
        c->u_copies_valid = false;
    }
    // the unitarity product too when steps check it, so that rtdm_step allocates nothing
    if (c->opt.unit_check_every > 0) schedule(c, RTDM_PROD_UV);
    RT_HIP(hipDeviceSynchronize());
    API_END(c)
}

int rtdm_pattern(rtdm_ctx *c, rtdm_mat mat, int64_t *n_rows, int64_t *nnzb, const int64_t **row_ptr,
                 const int32_t **col_idx)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    require(c->ranges_set, "set_ranges first");
    RT_CHECK(mat >= 0 && mat < RTDM_MAT_COUNT, RTDM_E_ARG, "bad matrix slot");
    const Pattern &P = pat_of(c, slot_range(mat));
    if (n_rows) *n_rows = P.n;
    if (nnzb) *nnzb = P.nnzb;
    if (row_ptr) *row_ptr = P.rowptr.data();
    if (col_idx) *col_idx = P.col.data();
    API_END(c)
}

namespace {

// Elements of block (i, j) in the caller's layout: b x b, or nbf_i x nbf_j
// (row-major) with mixed block sizes.
inline int64_t api_block_elems(const rtdm_ctx *c, int32_t i, int32_t j)
{
    return c->mixed ? (int64_t)c->nbf[i] * c->nbf[j] : (int64_t)c->b * c->b;
}

// Block t of the caller's data (starting at element offset `at`) into the
// padded b x b block at slot position p.
void put_block(const rtdm_ctx *c, int32_t i, int32_t j, const double *d, int64_t at, bool is_complex, int64_t p,
               std::vector<double> &re, std::vector<double> *im)
{
    const int b = c->b;
    const int ni = c->mixed ? c->nbf[i] : b, nj = c->mixed ? c->nbf[j] : b;
    for (int r = 0; r < ni; ++r)
        for (int q = 0; q < nj; ++q) {
            const int64_t src = at + (int64_t)r * nj + q, dst = p * b * b + (int64_t)r * b + q;
            if (is_complex) {
                re[dst] = d[2 * src];
                const double v = d[2 * src + 1];
                if (im) (*im)[dst] = v;
                else RT_CHECK(v == 0.0, RTDM_E_UNSUPPORTED, "complex data for a real matrix slot");
            } else {
                re[dst] = d[src];
            }
        }
}

// S and its inverse carry the identity on padded functions, so that these
// stay decoupled from the atom's own functions through every product.
void pad_identity(const rtdm_ctx *c, int mat, const Pattern &P, std::vector<double> &re)
{
    if (!c->mixed || (mat != RTDM_MAT_S && mat != RTDM_MAT_X)) return;
    const int b = c->b;
    for (int64_t i = 0; i < c->n; ++i) {
        auto b0 = P.col.begin() + P.rowptr[i], b1 = P.col.begin() + P.rowptr[i + 1];
        auto it = std::lower_bound(b0, b1, (int32_t)i);
        RT_CHECK(it != b1 && *it == i, RTDM_E_STATE, "pattern without its diagonal block");
        const int64_t p = it - P.col.begin();
        for (int a = c->nbf[i]; a < b; ++a) re[p * b * b + (int64_t)a * b + a] = 1.0;
    }
}

}  // namespace

int rtdm_upload(rtdm_ctx *c, rtdm_mat mat, const void *data, int is_complex, int is_device, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set, "set_ranges first");
    RT_CHECK(mat >= 0 && mat < RTDM_MAT_COUNT && data, RTDM_E_ARG, "bad upload arguments");
    hipStream_t s = (hipStream_t)stream;
    Mat &M = c->mats[mat];
    const int64_t ne = elems(c, M);
    RT_CHECK(!(c->mixed && is_device), RTDM_E_UNSUPPORTED, "device uploads need equal block sizes");
    if (!is_device && c->mixed) {
        // blocks of their own sizes, in pattern order
        const Pattern &P = *c->pats[M.pat];
        std::vector<double> re(ne, 0.0), im;
        if (M.cplx) im.assign(ne, 0.0);
        int64_t at = 0;
        for (int64_t i = 0; i < c->n; ++i)
            for (int64_t p = P.rowptr[i]; p < P.rowptr[i + 1]; ++p) {
                put_block(c, (int32_t)i, P.col[p], (const double *)data, at, is_complex, p, re, M.cplx ? &im : nullptr);
                at += api_block_elems(c, (int32_t)i, P.col[p]);
            }
        pad_identity(c, mat, P, re);
        upload_planes(c, mat, re.data(), M.cplx ? im.data() : nullptr, s);
    } else if (!is_device) {
        const double *d = (const double *)data;
        if (!is_complex) {
            upload_planes(c, mat, d, nullptr, s);
        } else {
            std::vector<double> re(ne), im(ne);
            bool nz = false;
            for (int64_t e = 0; e < ne; ++e) {
                re[e] = d[2 * e];
                im[e] = d[2 * e + 1];
                nz |= im[e] != 0.0;
            }
            RT_CHECK(M.cplx || !nz, RTDM_E_UNSUPPORTED, "complex data for a real matrix slot");
            upload_planes(c, mat, re.data(), im.data(), s);
        }
    } else {
        const double *d = (const double *)data;
        if (!is_complex) {
            RT_HIP(hipMemcpyAsync(M.re.p, d, ne * sizeof(double), hipMemcpyDeviceToDevice, s));
            if (M.cplx) RT_HIP(hipMemsetAsync(M.im.p, 0, M.im.bytes(), s));
        } else if (M.cplx) {
            launch_split(s, ne, d, M.re.p, M.im.p);
        } else {
            DBuf<double> tmp;
            tmp.alloc(ne);
            launch_split(s, ne, d, M.re.p, tmp.p);
            launch_red_sumsq(s, ne, tmp.p, c->partials.p);
            reduce_finish(c, s, c->hot_sums.p);
            double h[4];
            read_scalars(h, c->hot_sums.p, 4, s);
            RT_CHECK(h[3] == 0.0, RTDM_E_UNSUPPORTED, "complex data for a real matrix slot");
        }
    }
    after_upload(c, mat);
    API_END(c)
}

int rtdm_upload_coo(rtdm_ctx *c, rtdm_mat mat, int64_t nnzb, const int32_t *rows, const int32_t *cols,
                    const void *data, int is_complex, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set, "set_ranges first");
    RT_CHECK(mat >= 0 && mat < RTDM_MAT_COUNT && nnzb >= 0 && (nnzb == 0 || (rows && cols && data)),
             RTDM_E_ARG, "bad upload arguments");
    Mat &M = c->mats[mat];
    const Pattern &P = *c->pats[M.pat];
    const int64_t bb = (int64_t)c->b * c->b;
    const int64_t ne = P.nnzb * bb;
    std::vector<double> re(ne, 0.0), im;
    if (M.cplx) im.assign(ne, 0.0);
    (void)bb;
    const double *d = (const double *)data;
    int64_t at = 0;
    for (int64_t t = 0; t < nnzb; ++t) {
        const int32_t i = rows[t], j = cols[t];
        RT_CHECK(i >= 0 && i < c->n && j >= 0 && j < c->n, RTDM_E_ARG, "block index out of range");
        auto b0 = P.col.begin() + P.rowptr[i], b1 = P.col.begin() + P.rowptr[i + 1];
        auto it = std::lower_bound(b0, b1, j);
        RT_CHECK(it != b1 && *it == j, RTDM_E_ARG,
                 "block (" + std::to_string(i) + "," + std::to_string(j) + ") is outside the range");
        put_block(c, i, j, d, at, is_complex, it - P.col.begin(), re, M.cplx ? &im : nullptr);
        at += api_block_elems(c, i, j);
    }
    pad_identity(c, mat, P, re);
    upload_planes(c, mat, re.data(), M.cplx ? im.data() : nullptr, (hipStream_t)stream);
    after_upload(c, mat);
    API_END(c)
}

int rtdm_download(rtdm_ctx *c, rtdm_mat mat, void *dst, int is_device, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set, "set_ranges first");
    RT_CHECK(mat >= 0 && mat < RTDM_MAT_COUNT && dst, RTDM_E_ARG, "bad download arguments");
    hipStream_t s = (hipStream_t)stream;
    Mat &M = mat == RTDM_MAT_K ? kmat(c, c->kick_sel) : c->mats[mat];
    const int64_t ne = elems(c, M);
    if (mat == RTDM_MAT_W && c->W_in_cm) {             // the step keeps W column-major
        transpose_into(c, c->Wc, M, s);
        c->W_in_cm = false;
    }
    RT_CHECK(!(c->mixed && is_device), RTDM_E_UNSUPPORTED, "device downloads need equal block sizes");
    if (is_device) {
        launch_interleave(s, ne, M.re.p, M.cplx ? M.im.p : nullptr, (double *)dst);
        RT_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<double> re(ne), im(M.cplx ? ne : 0);
        RT_HIP(hipMemcpyAsync(re.data(), M.re.p, ne * sizeof(double), hipMemcpyDeviceToHost, s));
        if (M.cplx) RT_HIP(hipMemcpyAsync(im.data(), M.im.p, ne * sizeof(double), hipMemcpyDeviceToHost, s));
        RT_HIP(hipStreamSynchronize(s));
        double *o = (double *)dst;
        if (c->mixed) {
            // each block cut to its own nbf_i x nbf_j size, in pattern order
            const Pattern &P = *c->pats[M.pat];
            const int b = c->b;
            int64_t at = 0;
            for (int64_t i = 0; i < c->n; ++i)
                for (int64_t p = P.rowptr[i]; p < P.rowptr[i + 1]; ++p) {
                    const int ni = c->nbf[i], nj = c->nbf[P.col[p]];
                    for (int r = 0; r < ni; ++r)
                        for (int q = 0; q < nj; ++q, ++at) {
                            const int64_t e = p * b * b + (int64_t)r * b + q;
                            o[2 * at] = re[e];
                            o[2 * at + 1] = M.cplx ? im[e] : 0.0;
                        }
                }
        } else {
            for (int64_t e = 0; e < ne; ++e) {
                o[2 * e] = re[e];
                o[2 * e + 1] = M.cplx ? im[e] : 0.0;
            }
        }
    }
    API_END(c)
}

int rtdm_apply_kick(rtdm_ctx *c, const double kappa[3], void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_K] && c->uploaded[RTDM_MAT_S], "upload S and K first");
    RT_CHECK(kappa && std::isfinite(kappa[0]) && std::isfinite(kappa[1]) && std::isfinite(kappa[2]),
             RTDM_E_ARG, "bad kick");
    hipStream_t s = (hipStream_t)stream;
    if (!c->q_ref_valid) {
        c->charges_valid = false;
        ensure_charges(c, s);
    }
    const Pattern &P = pat_of(c, R_K);
    for (int k = 0; k < n_kicks(c); ++k)
        launch_kick(s, P.nnzb, c->b, P.d_rowof.p, P.d_col.p, c->d_xyz.p, kappa[0], kappa[1], kappa[2],
                    kmat(c, k).re.p, kmat(c, k).im.p);
    c->charges_valid = false;
    c->obs_rows = 0;
    c->obs_reset_pending = true;
    c->t_now = 0.0;
    c->step_count = 0;
    c->trace_dt_mixed = false;
    c->herm_valid = false;
    API_END(c)
}

int rtdm_build_inverse(rtdm_ctx *c, void *stream, int *iters, double *residual)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_S], "upload S first");
    hipStream_t s = (hipStream_t)stream;
    Mat &S = c->mats[RTDM_MAT_S];
    Mat &X = c->mats[RTDM_MAT_X];
    const Pattern &ps = pat_of(c, R_HS), &pp = pat_of(c, R_P);
    const int64_t ne = elems(c, X);

    auto start_block_jacobi = [&]() {
        RT_HIP(hipMemsetAsync(X.re.p, 0, X.re.bytes(), s));
        launch_block_inverse(s, c->n, c->b, ps.d_diag.p, S.re.p, pp.d_diag.p, X.re.p, c->scratch.p);
    };
    auto start_cold = [&]() {
        launch_row_abs_max(s, c->n, c->b, ps.d_rowptr.p, S.re.p, c->atom_max.p);
        launch_red_max(s, c->n, c->atom_max.p, c->partials.p);
        reduce_finish(c, s, c->hot_sums.p);
        double h[4];
        read_scalars(h, c->hot_sums.p, 4, s);
        RT_CHECK(h[3] > 0.0 && std::isfinite(h[3]), RTDM_E_NUMERIC, "S has no non-zero row");
        RT_HIP(hipMemsetAsync(X.re.p, 0, X.re.bytes(), s));
        launch_add_identity(s, c->n, c->b, pp.d_diag.p, 1.0 / h[3], X.re.p);
    };
    // On the b = 13 column-major path both products run on the step kernels:
    // a column-major copy of S (a context buffer, so the iteration allocates
    // nothing) for the whole iteration, of X per iteration.
    const bool cm = use_cm(c);
    Mat &Sc = c->Sc;
    if (cm) transpose_into(c, S, Sc, s);
    // X moves between buffers below and Xc is used as scratch: a captured step
    // that reads either must be captured again
    drop_graph(c);
    // Returns 1 converged, 0 diverged, -1 hit the cap.
    auto run = [&](int &k_out, double &r_out) -> int {
        std::vector<double> res;
        for (int k = 0; k < c->opt.inv_max_iter; ++k) {
            if (cm) {
                product_cm(c, RTDM_PROD_SX, Sc, X, c->Wh, 0, 0, 1.0, s);  // W = P_P(S X)
                transpose_into(c, X, c->Xc, s);
                product_cm(c, RTDM_PROD_AT, c->Xc, c->Wh, c->Xn, 0, 0, 1.0, s);   // P_P(X W)
            } else {
                product(c, RTDM_PROD_SX, S, X, c->Wh, 1.0, 0.0, s);       // W = P_P(S X)
                product(c, RTDM_PROD_AT, X, c->Wh, c->Xn, 1.0, 0.0, s);   // P_P(X W)
            }
            launch_axpby(s, ne, 2.0, X.re.p, -1.0, c->Xn.re.p, c->Xn.re.p);  // X' = 2X - XW
            launch_red_diff2(s, ne, c->Xn.re.p, X.re.p, c->partials.p);
            reduce_finish(c, s, c->hot_sums.p);
            double h[4];
            read_scalars(h, c->hot_sums.p, 4, s);
            // ||X'||^2 without the padded identity's ones (exactly n_pad of them)
            const double r = std::sqrt(h[0] / (h[1] - (double)c->n_pad));
            res.push_back(r);
            k_out = k + 1;
            r_out = r;
            if (!std::isfinite(r) || (k >= 1 && r > res[res.size() - 2])) return 0;
            std::swap(X.re, c->Xn.re);
            if (r <= c->opt.inv_tol) return 1;
        }
        return -1;
    };
    auto start_learned = [&]() {
        MlpState &M = c->mlp;
        RT_CHECK(M.ready && M.b == c->b, RTDM_E_STATE, "no trained network for the learned start");
        const int64_t n = ps.nnzb;
        // descriptors and predictions live in the A and U planes, which the
        // next step recomputes (U is marked stale below): no temporaries
        Mat &Am = c->mats[RTDM_MAT_A], &Um = c->mats[RTDM_MAT_U];
        RT_CHECK(Am.re.n * 2 >= (size_t)n * M.in && Um.re.n * 2 >= (size_t)n * M.out, RTDM_E_STATE,
                 "learned start: work planes too small");
        float *desc_p = reinterpret_cast<float *>(Am.re.p), *y_p = reinterpret_cast<float *>(Um.re.p);
        c->U_valid = false;
        const double inv_r = c->radius[R_HS] > 0 ? 1.0 / c->radius[R_HS] : 1.0;
        launch_mlp_desc(s, n, c->b, c->hs_iota.p, ps.d_rowof.p, ps.d_col.p, c->d_xyz.p, S.re.p, inv_r, desc_p);
        launch_mlp_forward(s, n, M.in, M.out, nullptr, desc_p, M.w1h.p, mlp_b1(M), M.w2h.p, mlp_b2(M),
                           nullptr, y_p);
        RT_HIP(hipMemsetAsync(X.re.p, 0, X.re.bytes(), s));
        launch_mlp_apply(s, n, c->b, c->hs_iota.p, c->hs_to_p.p, ps.d_rowof.p, ps.d_col.p, S.re.p, y_p, X.re.p);
        RT_HIP(hipStreamSynchronize(s));
    };
    int k = 0;
    double r = 0.0;
    int st;
    c->inv_fell_back = 0;
    if ((c->opt.inv_start == RTDM_INV_PREVIOUS && c->X_valid) || c->opt.inv_start == RTDM_INV_LEARNED) {
        if (c->opt.inv_start == RTDM_INV_LEARNED) start_learned();
        st = run(k, r);
        c->inv_iters_total = k;
        if (st != 1) {
            c->inv_fell_back = 1;
            start_block_jacobi();
            st = run(k, r);
            c->inv_iters_total += k;
        }
    } else {
        if (c->opt.inv_start == RTDM_INV_COLD) start_cold();
        else start_block_jacobi();
        st = run(k, r);
        c->inv_iters_total = k;
    }
    if (iters) *iters = k;
    if (residual) *residual = r;
    c->X_valid = (st == 1);
    c->Xc_valid = false;
    if (cm && st == 1) {
        transpose_into(c, X, c->Xc, s);   // the column-major copy of the converged X
        c->Xc_valid = true;
    }
    c->U_valid = false;
    c->A0_valid = false;
    RT_CHECK(st == 1, RTDM_E_NOCONV,
             "Hotelling iteration " + std::string(st == 0 ? "diverged" : "hit the iteration cap") +
                 " (residual " + std::to_string(r) + ")");
    API_END(c)
}

namespace {

bool h_varies(rtdm_ctx *c) { return c->opt.h_model == RTDM_HMODEL_MULLIKEN || c->field_on; }

// Kernel copy of both planes (graph-safe).
void copy_mat(rtdm_ctx *c, const Mat &src, Mat &dst, hipStream_t s)
{
    const int64_t ne = elems(c, src);
    launch_axpby(s, ne, 1.0, src.re.p, 0.0, nullptr, dst.re.p);
    if (dst.cplx) {
        if (src.cplx) launch_axpby(s, ne, 1.0, src.im.p, 0.0, nullptr, dst.im.p);
        else launch_fill(s, ne, 0.0, dst.im.p);
    }
}

// H(t + theta dt) into H: H0, the on-site term of the charges at that time
// point (extrapolated from q(t - dt), q(t); or, in a corrector pass,
// interpolated towards the q(t + dt) of the previous pass), and the field.
void build_h(rtdm_ctx *c, double theta, bool corr, hipStream_t s)
{
    Mat &H = c->mats[RTDM_MAT_H], &H0 = c->mats[RTDM_MAT_H0];
    const Pattern &ps = pat_of(c, R_HS);
    launch_axpby(s, elems(c, H), 1.0, H0.re.p, 0.0, nullptr, H.re.p);
    if (c->opt.h_model == RTDM_HMODEL_MULLIKEN) {
        if (corr)
            launch_onsite_shift(s, c->n, c->b, ps.d_diag.p, c->mixed ? c->d_nbf.p : nullptr, c->opt.h_gain, c->q_cur, theta, c->q_c.p, c->q_cur,
                                c->q_ref.p, H.re.p);
        else
            launch_onsite_shift(s, c->n, c->b, ps.d_diag.p, c->mixed ? c->d_nbf.p : nullptr, c->opt.h_gain, c->q_cur, theta, c->q_cur, c->q_prev,
                                c->q_ref.p, H.re.p);
    }
    if (c->field_on)
        launch_field(s, ps.nnzb, c->b, ps.d_rowof.p, ps.d_col.p, c->d_xyz.p, c->n_groups > 1 ? c->d_group.p : nullptr,
                     c->d_centre.p, c->mats[RTDM_MAT_S].re.p, c->field_E0, c->field_t0, c->field_sigma,
                     c->step_st.p, c->step_tt.p, theta, H.re.p);
}

// The Mulliken model without a field and with FP64 products forms A from
// A0 = P(X H0) and a column scaling of X (k_a_onsite): one product less per
// time point of a step.
bool a_from_a0(const rtdm_ctx *c)
{
    return c->opt.h_model == RTDM_HMODEL_MULLIKEN && !c->opt.xh_every_step && !c->field_on && c->A0.re.p != nullptr &&
           all_products_prec(const_cast<rtdm_ctx *>(c)) == RTDM_PREC_FP64;
}

// The column-major copy of X on the b = 13 path, refreshed when X changed.
// rtdm_step calls it before its steps, outside any capture: a captured step
// holds no transpose of X, so a graph replayed after X was replaced reads
// the copy made here.
void ensure_xc(rtdm_ctx *c, hipStream_t s)
{
    if (c->b != 13 || c->Xc_valid || !c->Xc.re.p) return;
    transpose_into(c, c->mats[RTDM_MAT_X], c->Xc, s);
    c->Xc_valid = true;
}

// A0 = P(X H0) for a_from_a0, built when X or H0 changed (outside any capture:
// rtdm_step calls it before its steps).
void ensure_a0(rtdm_ctx *c, hipStream_t s)
{
    if (!a_from_a0(c) || c->A0_valid) return;
    Mat &X = c->mats[RTDM_MAT_X], &H0 = c->mats[RTDM_MAT_H0];
    const int saved = c->prec;
    c->prec = RTDM_PREC_FP64;
    if (use_cm(c)) {
        ensure_xc(c, s);
        product_cm(c, RTDM_PROD_XH, c->Xc, H0, c->A0, 0, 0, 1.0, s);
    } else {
        product(c, RTDM_PROD_XH, X, H0, c->A0, 1.0, 0.0, s);
    }
    c->prec = saved;
    c->A0_valid = true;
}

// A = P_P(X H(t + theta dt)) (and its column-major copy on the b = 13 path).
void make_a(rtdm_ctx *c, double theta, bool corr, hipStream_t s)
{
    Mat &H = c->mats[RTDM_MAT_H], &X = c->mats[RTDM_MAT_X], &A = c->mats[RTDM_MAT_A];
    if (a_from_a0(c)) {
        RT_CHECK(c->A0_valid, RTDM_E_STATE, "A0 = P(X H0) not built before the step");
        const Pattern &pp = pat_of(c, R_P);
        launch_a_onsite(s, pp.nnzb, c->b, pp.d_col.p, c->mixed ? c->d_nbf.p : nullptr, c->opt.h_gain, c->q_cur,
                        theta, corr ? c->q_c.p : c->q_cur, corr ? c->q_cur : c->q_prev, c->q_ref.p, c->A0.re.p,
                        X.re.p, A.re.p);
        if (use_cm(c)) transpose_into(c, A, c->Ac, s);
        return;
    }
    build_h(c, theta, corr, s);
    if (use_cm(c)) {
        if (!c->Xc_valid) {
            transpose_into(c, X, c->Xc, s);
            c->Xc_valid = true;
        }
        product_cm(c, RTDM_PROD_XH, c->Xc, H, A, 0, 0, 1.0, s);
        transpose_into(c, A, c->Ac, s);
    } else {
        product(c, RTDM_PROD_XH, X, H, A, 1.0, 0.0, s);
    }
}

// The step's propagator U (and its column-major copy) for the options'
// scheme; corr selects interpolated charges (a corrector pass).
void build_u(rtdm_ctx *c, double dt, bool corr, hipStream_t s)
{
    Mat &A = c->mats[RTDM_MAT_A], &U = c->mats[RTDM_MAT_U];
    switch (c->opt.propagator) {
    case RTDM_PROP_EM:
        make_a(c, 0.5, corr, s);
        build_propagator(c, dt, s);
        break;
    case RTDM_PROP_ETRS:
        // U = P_P(exp(-i dt/2 A(1)) exp(-i dt/2 A(0)))
        make_a(c, 0.0, corr, s);
        build_propagator(c, 0.5 * dt, s);
        copy_mat(c, U, c->E1, s);
        make_a(c, 1.0, corr, s);
        build_propagator(c, 0.5 * dt, s);
        product(c, RTDM_PROD_AT, U, c->E1, c->E2, 1.0, 0.0, s);
        copy_mat(c, c->E2, U, s);
        if (use_cm(c)) transpose_into(c, U, c->Uc, s);
        break;
    case RTDM_PROP_M4: {
        // M = -i dt/2 (A1 + A2) - (sqrt(3) dt^2 / 12) (P(A2 A1) - P(A1 A2)), U = sum_n M^n / n!
        const double th1 = 0.5 - std::sqrt(3.0) / 6.0, th2 = 0.5 + std::sqrt(3.0) / 6.0;
        const int64_t ne = elems(c, A);
        make_a(c, th1, corr, s);
        copy_mat(c, A, c->A1, s);
        make_a(c, th2, corr, s);                                              // A = A2
        product(c, RTDM_PROD_AT, A, c->A1, c->tau[0], 1.0, 0.0, s);           // A2 A1
        product(c, RTDM_PROD_AT, c->A1, A, c->tau[1], 1.0, 0.0, s);           // A1 A2
        launch_axpby(s, ne, 1.0, c->tau[0].re.p, -1.0, c->tau[1].re.p, c->tau[0].re.p);
        launch_axpby(s, ne, -std::sqrt(3.0) * dt * dt / 12.0, c->tau[0].re.p, 0.0, nullptr, c->E1.re.p);
        launch_axpby(s, ne, 1.0, c->A1.re.p, 1.0, A.re.p, c->E1.im.p);
        launch_axpby(s, ne, -0.5 * dt, c->E1.im.p, 0.0, nullptr, c->E1.im.p);
        launch_fill(s, ne, 0.0, U.re.p);
        launch_fill(s, ne, 0.0, U.im.p);
        launch_add_identity(s, c->n, c->b, pat_of(c, R_P).d_diag.p, 1.0, U.re.p);
        const int p = c->opt.taylor_order;
        if (p >= 1) {
            launch_axpby(s, ne, 1.0, U.re.p, 1.0, c->E1.re.p, U.re.p);
            launch_axpby(s, ne, 1.0, U.im.p, 1.0, c->E1.im.p, U.im.p);
        }
        const Mat *prev = &c->E1;
        Mat *bufs[2] = {&c->E2, &c->E3};
        for (int k = 2; k <= p; ++k) {
            Mat &next = *bufs[k % 2];
            product(c, RTDM_PROD_AT, c->E1, *prev, next, 1.0 / k, 0.0, s);   // T_k = P(M T_{k-1}) / k
            launch_axpby(s, ne, 1.0, U.re.p, 1.0, next.re.p, U.re.p);
            launch_axpby(s, ne, 1.0, U.im.p, 1.0, next.im.p, U.im.p);
            prev = &next;
        }
        if (use_cm(c)) transpose_into(c, U, c->Uc, s);
        break;
    }
    default: throw Error(RTDM_E_ARG, "unknown propagator");
    }
    if (c->Uh_on) {
        const Pattern &pp = pat_of(c, R_P);
        launch_conj_transpose(s, pp.nnzb, c->b, pp.d_trans.p, U.re.p, U.im.p, c->Uh.re.p, c->Uh.im.p);
    }
    c->u_copies_valid = true;
}

// After an upload of U: its column-major copy (b = 13) and U^dagger (b = 4),
// made before the steps, outside any capture, since a step that keeps U
// (fixed H) does not rebuild them.
void ensure_u_copies(rtdm_ctx *c, hipStream_t s)
{
    if (c->u_copies_valid || !c->U_valid) return;
    Mat &U = c->mats[RTDM_MAT_U];
    const int saved = c->prec;
    c->prec = all_products_prec(c);
    if (use_cm(c)) transpose_into(c, U, c->Uc, s);
    c->prec = saved;
    if (c->Uh_on) {
        const Pattern &pp = pat_of(c, R_P);
        launch_conj_transpose(s, pp.nnzb, c->b, pp.d_trans.p, U.re.p, U.im.p, c->Uh.re.p, c->Uh.im.p);
    }
    c->u_copies_valid = true;
}

// One step on stream s: `passes` propagations of the same K(t) (the first
// with extrapolated charges, the others corrector passes), then the
// observables of the new K.  Everything here is a kernel launch (no memset
// or memcpy), so the same sequence can be captured into a HIP graph and
// replayed; the trace row and the time come from the device step state.
void step_body(rtdm_ctx *c, double dt, bool rebuild_u, int passes, hipStream_t s)
{
    Mat &U = c->mats[RTDM_MAT_U], &W = c->mats[RTDM_MAT_W];
    const Pattern &ps = pat_of(c, R_HS), &pk = pat_of(c, R_K);
    const int NK = n_kicks(c);                   // several kicks: fixed H, no corrector (checked at creation)
    c->prec = all_products_prec(c);
    const bool sc = passes > 1;
    for (int kk = 0; kk < NK; ++kk) {
        Mat &K = kmat(c, kk);
        Mat &dst = sc ? c->Kt : K;
        for (int it = 0; it < passes; ++it) {
            if (rebuild_u && kk == 0) {          // every kick shares the step's propagator
                build_u(c, dt, it > 0, s);
                c->U_valid = true;
                c->U_dt = dt;
            }
            if (use_cm(c)) {
                product_cm(c, RTDM_PROD_UK, c->Uc, K, c->Wc, 0, 1, 1.0, s);     // W, column-major
                product_cm(c, RTDM_PROD_WU, c->Wc, c->Uc, c->Kn, 1, 0, 1.0, s); // B = U^dagger
                c->W_in_cm = true;
            } else {
                product(c, RTDM_PROD_UK, U, K, W, 1.0, 0.0, s);
                if (c->Uh_on) product_key(c, RTDM_PROD_WU, wuh_key(c), W, c->Uh, c->Kn, 1.0, 0.0, s);
                else product(c, RTDM_PROD_WU, W, U, c->Kn, 1.0, 0.0, s);
                c->W_in_cm = false;
            }
            launch_hermitize(s, pk.nnzb, c->b, pk.d_trans.p, c->Kn.re.p, c->Kn.im.p, dst.re.p, dst.im.p,
                             c->partials.p);
            if (sc)
                launch_mulliken(s, c->n, c->b, ps.d_rowptr.p, ps.d_trans.p, c->s_to_k.p,
                                c->mats[RTDM_MAT_S].re.p, dst.re.p, c->q_c.p);
        }
        reduce_finish(c, s, herm_of(c, kk));
    }
    c->herm_valid = true;
    launch_axpby(s, c->n * NK, 1.0, c->q_cur, 0.0, nullptr, c->q_prev);            // q(t - dt) <- q(t)
    if (sc) {
        copy_mat(c, c->Kt, c->mats[RTDM_MAT_K], s);
        launch_axpby(s, c->n, 1.0, c->q_c.p, 0.0, nullptr, c->q_cur);
    } else {
        for (int kk = 0; kk < NK; ++kk)
            launch_mulliken(s, c->n, c->b, ps.d_rowptr.p, ps.d_trans.p, c->s_to_k.p, c->mats[RTDM_MAT_S].re.p,
                            kmat(c, kk).re.p, qcur(c, kk));
    }
    for (int kk = 0; kk < NK; ++kk) {
        launch_observables_step(s, c->n, c->d_xyz.p, c->d_centre_all.p, qcur(c, kk), herm_of(c, kk), obs_of(c, kk),
                                c->step_st.p, c->step_tt.p);
        if (c->n_groups > 1)
            launch_group_obs(s, c->n_groups, c->d_gptr.p, c->d_xyz.p, c->d_centre.p, qcur(c, kk), c->step_st.p,
                             obs_g_of(c, kk));
    }
    launch_step_end(s, c->step_st.p);
    c->prec = RTDM_PREC_FP64;
}

}  // namespace

namespace {

// Host side of one rtdm_step (or rtdm_batch_step) call on one context.
struct StepCall {
    rtdm_ctx *c;
    double dt;
    int64_t n_steps;
    hipStream_t s;
    double t_start;
    bool vary;
    int64_t k = 0;   // steps done in this call
};

void step_ready(rtdm_ctx *c, double dt, int64_t n_steps)
{
    require(c->ranges_set && c->X_valid && c->uploaded[RTDM_MAT_K] && c->uploaded[RTDM_MAT_H0] &&
                c->uploaded[RTDM_MAT_S],
            "upload S, H0, K and build (or upload) the inverse first");
    RT_CHECK(std::isfinite(dt) && n_steps >= 0, RTDM_E_ARG, "bad step arguments");
}

// Trace room, charges and the device step state for n_steps more steps.
StepCall step_begin(rtdm_ctx *c, double dt, int64_t n_steps, hipStream_t s)
{
    ensure_obs(c, c->obs_rows + n_steps);
    ensure_charges(c, s);
    ensure_xc(c, s);
    ensure_a0(c, s);
    ensure_u_copies(c, s);
    if (c->obs_reset_pending) {
        RT_HIP(hipMemsetAsync(c->step_st.p, 0, c->step_st.bytes(), s));
        c->obs_reset_pending = false;
    }
    launch_step_begin(s, c->step_st.p, c->step_tt.p, c->t_now, dt);
    return StepCall{c, dt, n_steps, s, c->t_now, h_varies(c)};
}

// Host bookkeeping after the step k of the call (and the unitarity check or
// monitor when one is due).
void after_step(StepCall &sc)
{
    rtdm_ctx *c = sc.c;
    hipStream_t s = sc.s;
    c->t_now = sc.t_start + (double)(sc.k + 1) * sc.dt;
    if (c->opt.unit_check_every > 0 && (c->obs_rows + 1) % c->opt.unit_check_every == 0) {
        c->prec = RTDM_PREC_FP64;               // the unitarity check stays FP64
        unitarity_sums(c, s);
        for (int kk = 0; kk < n_kicks(c); ++kk)   // U is shared: the same value in every kick's trace
            launch_unit_to_row(s, c->unit_sums.p, c->s_norm2.p, obs_of(c, kk) + 8 * c->obs_rows);
        if (c->opt.unit_tol > 0.0) {             // monitor: one synchronising read per check
            double row[8];
            read_scalars(row, c->obs.p + 8 * c->obs_rows, 8, s);
            const bool bad = !std::isfinite(row[4]) || !std::isfinite(row[6]) || row[6] > c->opt.unit_tol;
            if (bad) {
                c->obs_rows++;
                c->step_count++;
                throw Error(RTDM_E_NUMERIC, "step " + std::to_string(c->step_count) + ": unitarity error " +
                                                std::to_string(row[6]) + " (tolerance " +
                                                std::to_string(c->opt.unit_tol) + ") or Tr(KS) " +
                                                std::to_string(row[4]));
            }
        }
    }
    if (c->obs_rows == 0) c->trace_dt = sc.dt;
    else if (sc.dt != c->trace_dt) c->trace_dt_mixed = true;
    c->obs_rows++;
    c->step_count++;
    sc.k++;
}

void eager_step(StepCall &sc)
{
    rtdm_ctx *c = sc.c;
    const bool sc_now = sc.vary && c->opt.sc_iters > 0 && c->step_count < c->opt.sc_steps;
    step_body(c, sc.dt, sc.vary || !c->U_valid || c->U_dt != sc.dt, sc_now ? 1 + c->opt.sc_iters : 1, sc.s);
    after_step(sc);
}

// Steps that cannot be replayed from a captured step: the one that builds a
// fixed H's propagator, and those with corrector passes after a kick.
void eager_prefix(StepCall &sc)
{
    rtdm_ctx *c = sc.c;
    while (sc.k < sc.n_steps && !sc.vary && (!c->U_valid || c->U_dt != sc.dt)) eager_step(sc);
    while (sc.k < sc.n_steps && sc.vary && c->opt.sc_iters > 0 && c->step_count < c->opt.sc_steps)
        eager_step(sc);
}

// Record `count` consecutive steps of every context into one graph: each
// context's steps on a stream of its own forked from s (capture mode
// thread-local), joined back into s at the end.
void capture_steps(const std::vector<StepCall *> &calls, const std::vector<hipStream_t> &branch,
                   const std::vector<hipEvent_t> &ev, int count, hipStream_t s, hipGraph_t &graph,
                   hipGraphExec_t &exec)
{
    const size_t n = calls.size();
    for (auto *sc : calls) sc->c->capturing = true;
    RT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        if (n == 1) {
            for (int j = 0; j < count; ++j) step_body(calls[0]->c, calls[0]->dt, calls[0]->vary, 1, s);
        } else {
            RT_HIP(hipEventRecord(ev[0], s));
            for (size_t i = 0; i < n; ++i) {
                RT_HIP(hipStreamWaitEvent(branch[i], ev[0], 0));
                for (int j = 0; j < count; ++j) step_body(calls[i]->c, calls[i]->dt, calls[i]->vary, 1, branch[i]);
                RT_HIP(hipEventRecord(ev[1 + i], branch[i]));
                RT_HIP(hipStreamWaitEvent(s, ev[1 + i], 0));
            }
        }
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(s, &g);
        if (g) (void)hipGraphDestroy(g);
        for (auto *sc : calls) sc->c->capturing = false;
        throw;
    }
    RT_HIP(hipStreamEndCapture(s, &graph));
    for (auto *sc : calls) sc->c->capturing = false;
    RT_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
}

}  // namespace

int rtdm_step(rtdm_ctx *c, double dt, int64_t n_steps, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    step_ready(c, dt, n_steps);
    hipStream_t s = (hipStream_t)stream;
    if (c->opt.use_graph && !s) {
        if (!c->gstream) RT_HIP(hipStreamCreate(&c->gstream));
        s = c->gstream;
    }
    StepCall sc = step_begin(c, dt, n_steps, s);
    eager_prefix(sc);
    if (sc.k < n_steps && c->opt.use_graph) {
        if (c->gexec && (c->graph_dt != dt || c->graph_rebuilds_u != sc.vary)) drop_graph(c);
        const std::vector<StepCall *> one{&sc};
        if (!c->gexec) {
            capture_steps(one, {}, {}, 1, s, c->graph, c->gexec);
            c->graph_dt = dt;
            c->graph_rebuilds_u = sc.vary;
        }
        // whole groups of graph_steps steps replay one multi-step graph (the
        // step state lives on the device, so the steps of one graph follow
        // each other as eager steps do); the unitarity monitor needs the host
        // between steps, so it keeps single-step replays
        const int G = c->opt.graph_steps;
        if (G > 1 && c->opt.unit_check_every == 0) {
            while (n_steps - sc.k >= G) {
                if (!c->gexec_multi) capture_steps(one, {}, {}, G, s, c->graph_multi, c->gexec_multi);
                RT_HIP(hipGraphLaunch(c->gexec_multi, s));
                for (int j = 0; j < G; ++j) after_step(sc);
            }
        }
        while (sc.k < n_steps) {
            RT_HIP(hipGraphLaunch(c->gexec, s));
            after_step(sc);
        }
    }
    while (sc.k < n_steps) eager_step(sc);
    API_END(c)
}

// ------------------------------------------------------------------ batches

struct rtdm_batch {
    std::vector<rtdm_ctx *> ctx;
    int device = 0;
    int graph_steps = 16;
    std::vector<hipStream_t> branch;   // one capture branch per context
    std::vector<hipEvent_t> ev;        // fork, then one join per context
    hipStream_t own = nullptr;         // the call's stream when the caller passes none (blocking)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> epochs;      // graph_epoch of every context at capture
    std::vector<char> varies;          // every context's H varied (U rebuilt each step) at capture
    double dt = 0.0;
    std::string err;
};

namespace {

static void batch_drop(rtdm_batch *bt)
{
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
}

}  // namespace

#define BATCH_BEGIN try {
#define BATCH_END(bt)                                             \
    }                                                             \
    catch (const rtdm::Error &e) {                                \
        (bt)->err = e.what();                                     \
        return e.code;                                            \
    }                                                             \
    catch (const std::bad_alloc &) {                              \
        (bt)->err = "host allocation failed";                     \
        return RTDM_E_OOM;                                        \
    }                                                             \
    catch (const std::exception &e) {                             \
        (bt)->err = e.what();                                     \
        return RTDM_E_ARG;                                        \
    }                                                             \
    (bt)->err.clear();                                            \
    return RTDM_OK;

int rtdm_batch_create(rtdm_batch **out, rtdm_ctx *const *ctxs, int n_ctx, int graph_steps)
{
    if (!out || !ctxs || n_ctx < 1 || n_ctx > 64 || graph_steps < 1 || graph_steps > 1024) return RTDM_E_ARG;
    *out = nullptr;
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i] || ctxs[i]->device != ctxs[0]->device) return RTDM_E_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return RTDM_E_ARG;
    }
    auto *bt = new (std::nothrow) rtdm_batch;
    if (!bt) return RTDM_E_OOM;
    bt->ctx.assign(ctxs, ctxs + n_ctx);
    bt->device = ctxs[0]->device;
    bt->graph_steps = graph_steps;
    if (hipSetDevice(bt->device) != hipSuccess) {
        delete bt;
        return RTDM_E_HIP;
    }
    bool ok = true;
    bt->branch.assign(n_ctx, nullptr);
    bt->ev.assign(n_ctx + 1, nullptr);
    for (auto &st : bt->branch) ok = ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (auto &e : bt->ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        rtdm_batch_destroy(bt);
        return RTDM_E_HIP;
    }
    *out = bt;
    return RTDM_OK;
}

int rtdm_batch_step(rtdm_batch *bt, double dt, int64_t n_steps, void *stream)
{
    if (!bt) return RTDM_E_ARG;
    BATCH_BEGIN
    RT_HIP(hipSetDevice(bt->device));
    hipStream_t s = (hipStream_t)stream;
    if (!s) {
        // blocking (ordered with the null stream), so that later null-stream calls see the steps
        if (!bt->own) RT_HIP(hipStreamCreate(&bt->own));
        s = bt->own;
    }
    for (auto *c : bt->ctx) {
        step_ready(c, dt, n_steps);
        RT_CHECK(c->opt.unit_check_every == 0, RTDM_E_UNSUPPORTED,
                 "batched steps need unit_check_every = 0 (the check runs between steps on the host)");
    }
    std::vector<StepCall> calls;
    calls.reserve(bt->ctx.size());
    for (auto *c : bt->ctx) {
        DevMemScope scope(&c->mem);
        calls.push_back(step_begin(c, dt, n_steps, s));
        eager_prefix(calls.back());
    }
    // the captured part starts where every context has done its eager steps
    int64_t k0 = 0;
    for (auto &sc : calls) k0 = std::max(k0, sc.k);
    for (auto &sc : calls) {
        DevMemScope scope(&sc.c->mem);
        while (sc.k < k0) eager_step(sc);
    }
    const int G = bt->graph_steps;
    if (n_steps - k0 >= G) {
        bool stale = !bt->exec || bt->dt != dt;
        for (size_t i = 0; i < calls.size() && !stale; ++i)
            stale = bt->epochs[i] != calls[i].c->graph_epoch || bt->varies[i] != (char)calls[i].vary;
        if (stale) {
            batch_drop(bt);
            std::vector<StepCall *> ptrs;
            for (auto &sc : calls) ptrs.push_back(&sc);
            capture_steps(ptrs, bt->branch, bt->ev, G, s, bt->graph, bt->exec);
            bt->dt = dt;
            bt->epochs.clear();
            bt->varies.clear();
            for (auto &sc : calls) {
                bt->epochs.push_back(sc.c->graph_epoch);
                bt->varies.push_back((char)sc.vary);
            }
        }
        while (n_steps - calls[0].k >= G) {
            RT_HIP(hipGraphLaunch(bt->exec, s));
            for (auto &sc : calls)
                for (int j = 0; j < G; ++j) after_step(sc);
        }
    }
    // the rest as eager steps (a captured graph of fewer steps would be used once)
    for (auto &sc : calls) {
        DevMemScope scope(&sc.c->mem);
        while (sc.k < n_steps) eager_step(sc);
    }
    BATCH_END(bt)
}

const char *rtdm_batch_last_error(const rtdm_batch *bt) { return bt ? bt->err.c_str() : "null batch"; }

int rtdm_batch_destroy(rtdm_batch *bt)
{
    if (!bt) return RTDM_OK;
    (void)hipSetDevice(bt->device);
    batch_drop(bt);
    for (auto st : bt->branch)
        if (st) (void)hipStreamDestroy(st);
    for (auto e : bt->ev)
        if (e) (void)hipEventDestroy(e);
    if (bt->own) (void)hipStreamDestroy(bt->own);
    delete bt;
    return RTDM_OK;
}

int rtdm_ground_state(rtdm_ctx *c, double n_occ, double tol, int max_iter, void *stream, int *iters_out,
                      double *idem_out, uint64_t *branches_out)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->X_valid && c->uploaded[RTDM_MAT_H0] && c->uploaded[RTDM_MAT_S],
            "upload S, H0 and build (or upload) the inverse first");
    RT_CHECK(!c->mixed, RTDM_E_UNSUPPORTED, "the ground state needs equal block sizes");
    RT_CHECK(n_occ > 0 && std::isfinite(n_occ) && tol > 0 && max_iter >= 1 && max_iter <= 64, RTDM_E_ARG,
             "bad ground-state arguments (max_iter 1..64)");
    hipStream_t s = (hipStream_t)stream;
    c->prec = RTDM_PREC_FP64;
    Mat &A = c->mats[RTDM_MAT_A], &X = c->mats[RTDM_MAT_X], &K = c->mats[RTDM_MAT_K];
    const Pattern &pp = pat_of(c, R_P), &pk = pat_of(c, R_K);
    const int64_t ne = elems(c, A);
    product(c, RTDM_PROD_XH, X, c->mats[RTDM_MAT_H0], A, 1.0, 0.0, s);
    // Gershgorin bounds of A: per element row, centre and radius; extremes on the host
    DBuf<double> lohi;
    lohi.alloc(2 * c->n * c->b);
    launch_gershgorin(s, c->n, c->b, pp.d_rowptr.p, pp.d_diag.p, A.re.p, lohi.p);
    std::vector<double> h(2 * c->n * c->b);
    RT_HIP(hipMemcpyAsync(h.data(), lohi.p, lohi.bytes(), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    double lo = h[0], hi = h[1];
    for (size_t e = 0; e < h.size(); e += 2) {
        lo = std::min(lo, h[e]);
        hi = std::max(hi, h[e + 1]);
    }
    RT_CHECK(hi > lo, RTDM_E_NUMERIC, "degenerate spectral bounds");
    // Z_0 = (hi I - A) / (hi - lo)
    Mat *Z = &c->tau[0], *Z2 = &c->tau[1];
    launch_axpby(s, ne, -1.0 / (hi - lo), A.re.p, 0.0, nullptr, Z->re.p);
    launch_add_identity(s, c->n, c->b, pp.d_diag.p, hi / (hi - lo), Z->re.p);
    double prev = 0.0, idem = 0.0;
    uint64_t branches = 0;
    int it = 0;
    bool done = false;
    for (; it < max_iter && !done; ++it) {
        product(c, RTDM_PROD_AT, *Z, *Z, *Z2, 1.0, 0.0, s);
        launch_red_trace(s, c->n, c->b, pp.d_diag.p, Z->re.p, c->partials.p);
        reduce_finish(c, s, c->hot_sums.p);
        launch_red_trace(s, c->n, c->b, pp.d_diag.p, Z2->re.p, c->partials.p);
        reduce_finish(c, s, c->obs_tmp.p);
        double tz, tz2;
        read_scalars(&tz, c->hot_sums.p, 1, s);
        read_scalars(&tz2, c->obs_tmp.p, 1, s);
        idem = std::fabs(tz - tz2);
        if (idem <= tol * n_occ || (it >= 1 && prev < 1e-4 * n_occ && idem >= prev)) {
            done = true;
            break;
        }
        prev = idem;
        if (tz > n_occ) {
            std::swap(Z, Z2);
        } else {
            launch_axpby(s, ne, 2.0, Z->re.p, -1.0, Z2->re.p, Z->re.p);
            branches |= uint64_t(1) << it;
        }
    }
    if (iters_out) *iters_out = done ? it + 1 : it;
    if (idem_out) *idem_out = idem;
    if (branches_out) *branches_out = branches;
    RT_CHECK(done, RTDM_E_NOCONV, "purification did not reach its idempotency tolerance");
    // K = (P_K(Z X) + P_K(Z X)^T) / 2
    product(c, RTDM_PROD_ZX, *Z, X, c->Kn, 1.0, 0.0, s);
    launch_fill(s, elems(c, c->Kn), 0.0, c->Kn.im.p);
    launch_hermitize(s, pk.nnzb, c->b, pk.d_trans.p, c->Kn.re.p, c->Kn.im.p, K.re.p, K.im.p, c->partials.p);
    RT_HIP(hipStreamSynchronize(s));
    after_upload(c, RTDM_MAT_K);
    API_END(c)
}

int rtdm_reserve_trace(rtdm_ctx *c, int64_t rows)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(rows >= 0 && rows <= (int64_t(1) << 32), RTDM_E_ARG, "rows outside 0..2^32");
    ensure_obs(c, rows);
    API_END(c)
}

int rtdm_workspace_size(rtdm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return RTDM_E_ARG;
    API_BEGIN
    size_t tot = 0;
    for (auto *b : c->mem.bufs) tot += devmem_align(b->nbytes);
    *bytes = tot + kWorkspaceReserve;
    API_END(c)
}

int rtdm_bind_workspace(rtdm_ctx *c, void *ptr, size_t bytes)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(ptr && (reinterpret_cast<uintptr_t>(ptr) & 255) == 0, RTDM_E_ARG,
             "the workspace must be a 256-byte aligned device pointer");
    RT_CHECK(!c->mem.base, RTDM_E_STATE, "a workspace is already bound");
    hipPointerAttribute_t attr;
    RT_CHECK(hipPointerGetAttributes(&attr, ptr) == hipSuccess && attr.type == hipMemoryTypeDevice &&
                 attr.device == c->device,
             RTDM_E_ARG, "the workspace is not device memory of the context's device");
    std::vector<DBufBase *> list(c->mem.bufs.begin(), c->mem.bufs.end());
    std::sort(list.begin(), list.end(), [](DBufBase *a, DBufBase *b) { return a->raw() < b->raw(); });
    size_t need = 0;
    for (auto *b : list) need += devmem_align(b->nbytes);
    RT_CHECK(need <= bytes, RTDM_E_OOM, "workspace too small: " + std::to_string(need) + " bytes needed");
    RT_HIP(hipDeviceSynchronize());
    drop_graph(c);
    const bool cur_a = c->q_cur == c->q_a.p;
    char *base = static_cast<char *>(ptr);
    size_t off = 0;
    for (auto *b : list) {
        void *np = base + off;
        RT_HIP(hipMemcpy(np, b->raw(), b->nbytes, hipMemcpyDeviceToDevice));
        if (b->ext) c->mem.ext_free(b->raw(), c->mem.ext_user);
        else RT_HIP(hipFree(b->raw()));
        b->set_raw(np);
        b->in_ws = true;
        b->ext = false;
        off += devmem_align(b->nbytes);
    }
    c->mem.base = base;
    c->mem.cap = bytes;
    c->mem.used = off;
    if (c->q_a.p) {
        c->q_cur = cur_a ? c->q_a.p : c->q_b.p;
        c->q_prev = cur_a ? c->q_b.p : c->q_a.p;
    }
    API_END(c)
}

int rtdm_set_allocator(rtdm_ctx *c, void *(*alloc_fn)(size_t, void *), void (*free_fn)(void *, void *),
                       void *user)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(alloc_fn && free_fn, RTDM_E_ARG, "null allocator functions");
    RT_CHECK(!c->mem.ext_alloc, RTDM_E_STATE, "the context already has an allocator");
    RT_CHECK(!c->mem.base, RTDM_E_STATE, "a workspace is bound");
    RT_HIP(hipDeviceSynchronize());
    drop_graph(c);
    const bool cur_a = c->q_cur == c->q_a.p;
    // move the buffers allocated so far into the caller's allocations
    std::vector<DBufBase *> list(c->mem.bufs.begin(), c->mem.bufs.end());
    std::vector<void *> homes(list.size(), nullptr);
    for (size_t k = 0; k < list.size(); ++k) {
        homes[k] = alloc_fn(list[k]->nbytes, user);
        if (!homes[k] || (reinterpret_cast<uintptr_t>(homes[k]) & 255) != 0) {
            for (void *h : homes)
                if (h) free_fn(h, user);
            throw Error(homes[k] ? RTDM_E_ARG : RTDM_E_OOM,
                        homes[k] ? "the allocator returned memory that is not 256-byte aligned"
                                 : "the allocator refused the context's buffers");
        }
    }
    for (size_t k = 0; k < list.size(); ++k) {
        RT_HIP(hipMemcpy(homes[k], list[k]->raw(), list[k]->nbytes, hipMemcpyDeviceToDevice));
        RT_HIP(hipFree(list[k]->raw()));
        list[k]->set_raw(homes[k]);
        list[k]->ext = true;
    }
    c->mem.ext_alloc = alloc_fn;
    c->mem.ext_free = free_fn;
    c->mem.ext_user = user;
    if (c->q_a.p) {
        c->q_cur = cur_a ? c->q_a.p : c->q_b.p;
        c->q_prev = cur_a ? c->q_b.p : c->q_a.p;
    }
    API_END(c)
}

int rtdm_unbind_workspace(rtdm_ctx *c)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(c->mem.base, RTDM_E_STATE, "no workspace is bound");
    RT_HIP(hipDeviceSynchronize());
    drop_graph(c);
    const bool cur_a = c->q_cur == c->q_a.p;
    std::vector<DBufBase *> list(c->mem.bufs.begin(), c->mem.bufs.end());
    // allocate every new home first, so that a failure leaves the context bound as it was
    std::vector<void *> homes(list.size(), nullptr);
    const bool ext = c->mem.ext_alloc != nullptr;
    auto give_back = [&]() {
        for (void *h : homes)
            if (h) {
                if (ext) c->mem.ext_free(h, c->mem.ext_user);
                else (void)hipFree(h);
            }
    };
    for (size_t k = 0; k < list.size(); ++k) {
        if (!list[k]->in_ws) continue;
        if (ext) {
            homes[k] = c->mem.ext_alloc(list[k]->nbytes, c->mem.ext_user);
        } else if (hipMalloc(&homes[k], list[k]->nbytes) != hipSuccess) {
            (void)hipGetLastError();
            homes[k] = nullptr;
        }
        if (!homes[k]) {
            give_back();
            throw Error(RTDM_E_OOM, "allocation failed while moving out of the workspace");
        }
    }
    for (size_t k = 0; k < list.size(); ++k) {
        if (!homes[k]) continue;
        RT_HIP(hipMemcpy(homes[k], list[k]->raw(), list[k]->nbytes, hipMemcpyDeviceToDevice));
        list[k]->set_raw(homes[k]);
        list[k]->in_ws = false;
        list[k]->ext = ext;
    }
    c->mem.base = nullptr;
    c->mem.cap = 0;
    c->mem.used = 0;
    if (c->q_a.p) {
        c->q_cur = cur_a ? c->q_a.p : c->q_b.p;
        c->q_prev = cur_a ? c->q_b.p : c->q_a.p;
    }
    API_END(c)
}

int rtdm_set_field(rtdm_ctx *c, const double E0[3], double t0, double sigma)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    RT_CHECK(E0 && std::isfinite(E0[0]) && std::isfinite(E0[1]) && std::isfinite(E0[2]) && std::isfinite(t0) &&
                 std::isfinite(sigma) && sigma > 0.0,
             RTDM_E_ARG, "bad field (sigma must be > 0)");
    for (int k = 0; k < 3; ++k) c->field_E0[k] = E0[k];
    c->field_t0 = t0;
    c->field_sigma = sigma;
    c->field_on = E0[0] != 0.0 || E0[1] != 0.0 || E0[2] != 0.0;
    c->U_valid = false;
    drop_graph(c);
    API_END(c)
}

int rtdm_spectrum(rtdm_ctx *c, int64_t group, const double P0[3], const double *kappa, double gamma,
                  int64_t n_omega, const double *omega, double *alpha, double *strength, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(P0 && n_omega >= 0 && (omega || n_omega == 0) && (alpha || n_omega == 0) && std::isfinite(gamma),
             RTDM_E_ARG, "bad spectrum arguments");
    RT_CHECK(group < c->n_groups && (group < 0 || c->n_groups > 1), RTDM_E_ARG, "no such group");
    RT_CHECK(c->obs_rows >= 1, RTDM_E_STATE, "no steps since the last kick");
    RT_CHECK(!c->trace_dt_mixed, RTDM_E_STATE, "the trace mixes step lengths");
    RT_CHECK(kappa || c->field_on, RTDM_E_STATE, "neither a kick nor a field");
    hipStream_t s = (hipStream_t)stream;
    if (n_omega == 0) return RTDM_OK;
    DBuf<double> om, al, st;
    om.alloc(n_omega);
    al.alloc(n_omega * 6);
    st.alloc(n_omega);
    RT_HIP(hipMemcpyAsync(om.p, omega, om.bytes(), hipMemcpyHostToDevice, s));
    const double *trace = group < 0 ? obs_of(c, c->kick_sel) : obs_g_of(c, c->kick_sel);
    const int64_t stride = group < 0 ? 8 : 4 * c->n_groups;
    const int64_t off = group < 0 ? 1 : 4 * group;
    launch_spectrum(s, n_omega, om.p, gamma, c->trace_dt, c->obs_rows, trace, stride, off, P0, kappa ? 1 : 0,
                    kappa ? kappa : c->field_E0, c->field_t0, c->field_sigma, al.p, st.p);
    RT_HIP(hipMemcpyAsync(alpha, al.p, al.bytes(), hipMemcpyDeviceToHost, s));
    if (strength) RT_HIP(hipMemcpyAsync(strength, st.p, st.bytes(), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    API_END(c)
}

int rtdm_set_groups(rtdm_ctx *c, int64_t n_groups, const int64_t *group_ptr)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set, "set_ranges first");
    RT_CHECK(n_groups >= 1 && group_ptr && group_ptr[0] == 0 && group_ptr[n_groups] == c->n, RTDM_E_ARG,
             "group_ptr must run from 0 to n_atoms");
    std::vector<int32_t> grp(c->n);
    for (int64_t g = 0; g < n_groups; ++g) {
        RT_CHECK(group_ptr[g + 1] > group_ptr[g], RTDM_E_ARG, "empty group");
        for (int64_t i = group_ptr[g]; i < group_ptr[g + 1]; ++i) grp[i] = (int32_t)g;
    }
    for (auto &P : c->pats)
        for (int64_t p = 0; p < P->nnzb; ++p)
            RT_CHECK(grp[P->rowof[p]] == grp[P->col[p]], RTDM_E_ARG,
                     "a kept pair crosses groups: place the groups further apart");
    RT_HIP(hipDeviceSynchronize());
    c->n_groups = n_groups;
    c->gptr.assign(group_ptr, group_ptr + n_groups + 1);
    c->d_gptr.alloc(n_groups + 1);
    c->d_group.alloc(c->n);
    RT_HIP(hipMemcpy(c->d_gptr.p, group_ptr, c->d_gptr.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(c->d_group.p, grp.data(), c->d_group.bytes(), hipMemcpyHostToDevice));
    std::vector<double> cen(3 * n_groups, 0.0);
    for (int64_t g = 0; g < n_groups; ++g) exact_centre(c->xyz, group_ptr[g], group_ptr[g + 1], &cen[3 * g]);
    c->d_centre.alloc(3 * n_groups);
    RT_HIP(hipMemcpy(c->d_centre.p, cen.data(), c->d_centre.bytes(), hipMemcpyHostToDevice));
    c->obs_g.release();
    c->obs_cap = 0;
    ensure_obs(c, std::max<int64_t>(c->obs_rows, 1024));
    drop_graph(c);
    API_END(c)
}

int rtdm_apply_kick_groups(rtdm_ctx *c, const double *kappa, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_K] && c->uploaded[RTDM_MAT_S], "upload S and K first");
    RT_CHECK(kappa, RTDM_E_ARG, "null kicks");
    for (int64_t e = 0; e < 3 * c->n_groups; ++e) RT_CHECK(std::isfinite(kappa[e]), RTDM_E_ARG, "bad kick");
    hipStream_t s = (hipStream_t)stream;
    if (!c->q_ref_valid) {
        c->charges_valid = false;
        ensure_charges(c, s);
    }
    const Pattern &P = pat_of(c, R_K);
    if (c->n_groups == 1) {
        for (int k = 0; k < n_kicks(c); ++k)
            launch_kick(s, P.nnzb, c->b, P.d_rowof.p, P.d_col.p, c->d_xyz.p, kappa[0], kappa[1], kappa[2],
                        kmat(c, k).re.p, kmat(c, k).im.p);
    } else {
        c->kick_g.alloc(3 * c->n_groups);
        RT_HIP(hipMemcpyAsync(c->kick_g.p, kappa, c->kick_g.bytes(), hipMemcpyHostToDevice, s));
        for (int k = 0; k < n_kicks(c); ++k)
            launch_kick_groups(s, P.nnzb, c->b, P.d_rowof.p, P.d_col.p, c->d_xyz.p, c->d_group.p, c->kick_g.p,
                               kmat(c, k).re.p, kmat(c, k).im.p);
        RT_HIP(hipStreamSynchronize(s));
    }
    c->charges_valid = false;
    c->obs_rows = 0;
    c->obs_reset_pending = true;
    c->t_now = 0.0;
    c->step_count = 0;
    c->trace_dt_mixed = false;
    c->herm_valid = false;
    API_END(c)
}

int rtdm_apply_kicks(rtdm_ctx *c, const double *kappa, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_K] && c->uploaded[RTDM_MAT_S], "upload S and K first");
    RT_CHECK(kappa, RTDM_E_ARG, "null kicks");
    for (int e = 0; e < 3 * n_kicks(c); ++e) RT_CHECK(std::isfinite(kappa[e]), RTDM_E_ARG, "bad kick");
    hipStream_t s = (hipStream_t)stream;
    if (!c->q_ref_valid) {
        c->charges_valid = false;
        ensure_charges(c, s);
    }
    const Pattern &P = pat_of(c, R_K);
    for (int k = 0; k < n_kicks(c); ++k)
        launch_kick(s, P.nnzb, c->b, P.d_rowof.p, P.d_col.p, c->d_xyz.p, kappa[3 * k], kappa[3 * k + 1],
                    kappa[3 * k + 2], kmat(c, k).re.p, kmat(c, k).im.p);
    c->charges_valid = false;
    c->obs_rows = 0;
    c->obs_reset_pending = true;
    c->t_now = 0.0;
    c->step_count = 0;
    c->trace_dt_mixed = false;
    c->herm_valid = false;
    API_END(c)
}

int rtdm_select_kick(rtdm_ctx *c, int k)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    RT_CHECK(k >= 0 && k < n_kicks(c), RTDM_E_ARG, "no such kick set");
    c->kick_sel = k;
    API_END(c)
}

int rtdm_group_trace(rtdm_ctx *c, double *out, int64_t max_rows, int64_t *rows)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(max_rows >= 0 && (out || max_rows == 0), RTDM_E_ARG, "bad trace buffer");
    RT_CHECK(c->n_groups > 1, RTDM_E_STATE, "no groups set");
    RT_HIP(hipDeviceSynchronize());
    const int64_t nr = std::min(max_rows, c->obs_rows);
    if (rows) *rows = c->obs_rows;
    if (nr > 0)
        RT_HIP(hipMemcpy(out, obs_g_of(c, c->kick_sel), nr * c->n_groups * 4 * sizeof(double),
                         hipMemcpyDeviceToHost));
    API_END(c)
}

namespace {
// Re-derive the processing order of every schedule (outputs and row runs) for
// row tiles of `tile` atoms.
void set_row_tile(rtdm_ctx *c, int tile)
{
    c->row_tile = tile;
    for (auto &kv : c->scheds) {
        Sched &S = *kv.second;
        const std::vector<int32_t> ord = tile_order(*c->pats[std::get<2>(kv.first)], tile, 1 << 30);
        if (!ord.empty())
            RT_HIP(hipMemcpy(S.order.p, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        for (auto &rr : S.runs) {
            const Runs &R = *rr.second;
            if (R.nch == 0) continue;
            const std::vector<int32_t> ro = run_order(R, tile);
            RT_HIP(hipMemcpy(R.order.p, ro.data(), ro.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        }
    }
}
}  // namespace

int rtdm_autotune(rtdm_ctx *c, void *stream, int *wpb_out, int *tile_out)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set, "set_ranges first");
    hipStream_t s = (hipStream_t)stream;
    if (c->b == 13) {
        const int wpbs[3] = {4, 8, 16}, tiles[3] = {64, 256, 1024};
        // events and the context's timing flag are restored however the sweep ends
        struct Guard {
            rtdm_ctx *c;
            bool timing;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            ~Guard()
            {
                c->timing = timing;
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
            }
        } guard{c, c->timing};
        RT_HIP(hipEventCreate(&guard.e0));
        RT_HIP(hipEventCreate(&guard.e1));
        hipEvent_t e0 = guard.e0, e1 = guard.e1;
        double best = 1e300;
        int bw = c->wpb, bt = c->row_tile;
        c->timing = false;
        for (int tile : tiles) {
            set_row_tile(c, tile);
            for (int w : wpbs) {
                c->wpb = w;
                product_cm(c, RTDM_PROD_UK, c->Uc, c->mats[RTDM_MAT_K], c->Wc, 0, 1, 1.0, s);   // warm-up
                RT_HIP(hipEventRecord(e0, s));
                product_cm(c, RTDM_PROD_UK, c->Uc, c->mats[RTDM_MAT_K], c->Wc, 0, 1, 1.0, s);
                product_cm(c, RTDM_PROD_AT, c->Ac, c->tau[0], c->tau[1], 0, 0, 1.0, s);
                RT_HIP(hipEventRecord(e1, s));
                RT_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                RT_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    bw = w;
                    bt = tile;
                }
            }
        }
        c->wpb = bw;
        set_row_tile(c, bt);
        c->W_in_cm = true;
        drop_graph(c);
    }
    if (wpb_out) *wpb_out = c->wpb;
    if (tile_out) *tile_out = c->row_tile;
    API_END(c)
}

int rtdm_observables(rtdm_ctx *c, double out[6], void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_K] && c->uploaded[RTDM_MAT_S], "upload S and K first");
    RT_CHECK(out, RTDM_E_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    ensure_charges(c, s);
    launch_observables(s, c->n, c->d_xyz.p, c->d_centre_all.p, qcur(c, c->kick_sel),
                       c->herm_valid ? herm_of(c, c->kick_sel) : nullptr, c->t_now, c->obs_tmp.p);
    double row[8];
    read_scalars(row, c->obs_tmp.p, 8, s);
    for (int k = 0; k < 5; ++k) out[k] = row[k + 1];
    out[5] = std::nan("");
    if (c->U_valid) {
        unitarity_sums(c, s);
        double u[4], s2[4];
        read_scalars(u, c->unit_sums.p, 4, s);
        read_scalars(s2, c->s_norm2.p, 4, s);
        out[5] = std::sqrt(u[0] / s2[0]);
    }
    for (int k = 0; k < 5; ++k)
        RT_CHECK(std::isfinite(out[k]), RTDM_E_NUMERIC, "non-finite observable: the propagation has blown up");
    API_END(c)
}

int rtdm_get_state(rtdm_ctx *c, double *out, int64_t n, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_K] && c->uploaded[RTDM_MAT_S], "upload S and K first");
    RT_CHECK(out && n == 2 + 3 * c->n, RTDM_E_ARG, "the state holds 2 + 3 n_atoms doubles");
    hipStream_t s = (hipStream_t)stream;
    ensure_charges(c, s);
    out[0] = c->t_now;
    out[1] = (double)c->step_count;
    RT_HIP(hipMemcpyAsync(out + 2, qcur(c, c->kick_sel), c->n * sizeof(double), hipMemcpyDeviceToHost, s));
    RT_HIP(hipMemcpyAsync(out + 2 + c->n, qprev(c, c->kick_sel), c->n * sizeof(double), hipMemcpyDeviceToHost, s));
    RT_HIP(hipMemcpyAsync(out + 2 + 2 * c->n, c->q_ref.p, c->n * sizeof(double), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    API_END(c)
}

int rtdm_set_state(rtdm_ctx *c, const double *in, int64_t n, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_K] && c->uploaded[RTDM_MAT_S], "upload S and K first");
    RT_CHECK(in && n == 2 + 3 * c->n, RTDM_E_ARG, "the state holds 2 + 3 n_atoms doubles");
    RT_CHECK(std::isfinite(in[0]) && in[1] >= 0 && in[1] == std::floor(in[1]), RTDM_E_ARG, "bad time or step count");
    hipStream_t s = (hipStream_t)stream;
    RT_CHECK(n_kicks(c) == 1, RTDM_E_UNSUPPORTED, "set_state restores a single kick");
    RT_HIP(hipMemcpyAsync(c->q_cur, in + 2, c->n * sizeof(double), hipMemcpyHostToDevice, s));
    RT_HIP(hipMemcpyAsync(c->q_prev, in + 2 + c->n, c->n * sizeof(double), hipMemcpyHostToDevice, s));
    RT_HIP(hipMemcpyAsync(c->q_ref.p, in + 2 + 2 * c->n, c->n * sizeof(double), hipMemcpyHostToDevice, s));
    RT_HIP(hipStreamSynchronize(s));
    c->t_now = in[0];
    c->step_count = (int64_t)in[1];
    c->charges_valid = true;
    c->q_ref_valid = true;
    c->obs_rows = 0;
    c->obs_reset_pending = true;
    c->trace_dt_mixed = false;
    c->herm_valid = false;
    c->U_valid = false;
    API_END(c)
}

int rtdm_dipole_trace(rtdm_ctx *c, double *out, int64_t max_rows, int64_t *rows)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(max_rows >= 0 && (out || max_rows == 0), RTDM_E_ARG, "bad trace buffer");
    RT_HIP(hipDeviceSynchronize());
    const int64_t nr = std::min(max_rows, c->obs_rows);
    if (rows) *rows = c->obs_rows;
    if (nr > 0) {
        std::vector<double> tmp(nr * 8);
        RT_HIP(hipMemcpy(tmp.data(), obs_of(c, c->kick_sel), tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t r = 0; r < nr; ++r)
            for (int k = 0; k < 7; ++k) out[7 * r + k] = tmp[8 * r + k];
    }
    API_END(c)
}

int rtdm_unitarity(rtdm_ctx *c, double out[3], void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->U_valid && c->uploaded[RTDM_MAT_S], "no propagator yet");
    RT_CHECK(out, RTDM_E_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    unitarity_sums(c, s);
    double u[4], s2[4];
    read_scalars(u, c->unit_sums.p, 4, s);
    read_scalars(s2, c->s_norm2.p, 4, s);
    out[0] = std::sqrt(u[0] / s2[0]);
    out[1] = u[1] / ((double)pat_of(c, R_P).nnzb * c->b * c->b);
    out[2] = u[3];
    API_END(c)
}

int rtdm_inverse_error(rtdm_ctx *c, double out[3], void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set && c->X_valid && c->uploaded[RTDM_MAT_S], "build or upload the inverse first");
    RT_CHECK(out, RTDM_E_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    product(c, RTDM_PROD_XH, c->mats[RTDM_MAT_X], c->mats[RTDM_MAT_S], c->Wh, 1.0, 0.0, s);
    const Pattern &pp = pat_of(c, R_P);
    launch_red_minus_identity(s, pp.nnzb, c->b, pp.d_rowof.p, pp.d_col.p, c->Wh.re.p, c->partials.p);
    reduce_finish(c, s, c->hot_sums.p);
    double h[4];
    read_scalars(h, c->hot_sums.p, 4, s);
    out[0] = h[1] / ((double)pp.nnzb * c->b * c->b);
    out[1] = h[3];
    out[2] = std::sqrt(h[0]);
    API_END(c)
}

namespace {

// A Mat whose planes are borrowed device memory (the static scratch): the
// pointers are detached before the DBufs are destroyed, so nothing is freed.
struct BorrowedMat {
    Mat m;
    BorrowedMat(int pat, bool cplx, double *re, double *im, size_t n)
    {
        m.pat = pat;
        m.cplx = cplx;
        m.re.p = re;
        m.re.n = n;
        m.im.p = cplx ? im : nullptr;
        m.im.n = cplx ? n : 0;
    }
    ~BorrowedMat()
    {
        m.re.p = m.im.p = nullptr;
        m.re.n = m.im.n = 0;
    }
};

// rtdm_multiply's body.  scratch null: the b = 13 column-major copies are
// allocated (and the call waits for the stream before freeing them);
// otherwise they are cut from scratch (cap bytes), nothing is allocated and
// the call returns without waiting.
void multiply(rtdm_ctx *c, rtdm_mat Cm, rtdm_mat Am, rtdm_mat Bm, int op_a, int op_b, double alr, double ali,
              hipStream_t s, double *scratch, size_t cap)
{
    require(c->ranges_set, "set_ranges first");
    RT_CHECK(Am >= 0 && Am < RTDM_MAT_COUNT && Bm >= 0 && Bm < RTDM_MAT_COUNT && Cm >= 0 &&
                 Cm < RTDM_MAT_COUNT && (op_a == 0 || op_a == 1) && (op_b == 0 || op_b == 1),
             RTDM_E_ARG, "bad multiply arguments");
    RT_CHECK(Cm != Am && Cm != Bm, RTDM_E_ARG, "output aliases an operand");
    Mat &A = c->mats[Am], &B = c->mats[Bm], &C = c->mats[Cm];
    const std::tuple<int, int, int, int, int> want{A.pat, B.pat, C.pat, op_a, op_b};
    int prod = -1;
    for (int q = 0; q < RTDM_PROD_COUNT; ++q)
        if (prod_key(c, q) == want) { prod = q; break; }
    RT_CHECK(prod >= 0, RTDM_E_UNSUPPORTED, "no product kind with these ranges and operations");
    RT_CHECK(!scratch || c->scheds.count(want), RTDM_E_STATE,
             "no schedule of this product kind yet (the allocation-free call builds none): call rtdm_multiply once");
    const bool cres = A.cplx || B.cplx || ali != 0.0;
    RT_CHECK(C.cplx || !cres, RTDM_E_UNSUPPORTED, "complex result for a real matrix slot");
    c->prec = all_products_prec(c);
    try {
        // The step products of the b = 13 column-major path run exactly as in a
        // step: column-major copies of A (and of B when it is conjugate-
        // transposed), the row-run kernels, and U K written column-major.
        const bool step_kind = prod == RTDM_PROD_XH || prod == RTDM_PROD_AT || prod == RTDM_PROD_UK ||
                               prod == RTDM_PROD_WU;
        if (use_cm(c) && step_kind && op_a == 0 && ali == 0.0) {
            const size_t bb = (size_t)c->b * c->b;
            const size_t na = c->pats[A.pat]->nnzb * bb, nbm = c->pats[B.pat]->nnzb * bb,
                         nc = c->pats[C.pat]->nnzb * bb;
            const bool ccm = prod == RTDM_PROD_UK;
            auto planes = [](const Mat &m) { return m.cplx ? 2 : 1; };
            // scratch layout: A's planes, then B's (conjugate-transposed B), then C's (U K), each 256-byte aligned
            const size_t al = 256 / sizeof(double);
            auto up = [&](size_t n) { return (n + al - 1) / al * al; };
            const size_t need = planes(A) * up(na) + (op_b ? planes(B) * up(nbm) : 0) + (ccm ? planes(C) * up(nc) : 0);
            std::unique_ptr<BorrowedMat> va, vb, vc;
            Mat Acm, Bcm, Ccm;
            Mat *pa = &Acm, *pb = &Bcm, *pc = &Ccm;
            if (scratch) {
                RT_CHECK(need * sizeof(double) <= cap, RTDM_E_ARG,
                         "operands too large for the static scratch: " + std::to_string(need * sizeof(double)) +
                             " bytes needed, " + std::to_string(cap) + " available");
                double *p = scratch;
                auto take = [&](size_t n) { double *q = p; p += up(n); return q; };
                double *ar = take(na), *ai = A.cplx ? take(na) : nullptr;
                va = std::make_unique<BorrowedMat>(A.pat, A.cplx, ar, ai, na);
                pa = &va->m;
                if (op_b) {
                    double *br = take(nbm), *bi = B.cplx ? take(nbm) : nullptr;
                    vb = std::make_unique<BorrowedMat>(B.pat, B.cplx, br, bi, nbm);
                    pb = &vb->m;
                }
                if (ccm) {
                    double *cr = take(nc), *ci = C.cplx ? take(nc) : nullptr;
                    vc = std::make_unique<BorrowedMat>(C.pat, C.cplx, cr, ci, nc);
                    pc = &vc->m;
                }
            } else {
                alloc_like(c, Acm, A);
                if (op_b) alloc_like(c, Bcm, B);
                if (ccm) alloc_like(c, Ccm, C);
            }
            transpose_into(c, A, *pa, s);
            const Mat *Bp = &B;
            if (op_b) {
                transpose_into(c, B, *pb, s);
                Bp = pb;
            }
            if (ccm) {
                product_cm(c, prod, *pa, *Bp, *pc, op_b, 1, alr, s);
                transpose_into(c, *pc, C, s);
            } else {
                product_cm(c, prod, *pa, *Bp, C, op_b, 0, alr, s);
            }
            if (!scratch) RT_HIP(hipStreamSynchronize(s));   // the copies are freed on return
        } else {
            product(c, prod, A, B, C, alr, ali, s);
        }
    } catch (...) {
        c->prec = RTDM_PREC_FP64;
        throw;
    }
    c->prec = RTDM_PREC_FP64;
    after_upload(c, Cm);
}

}  // namespace

int rtdm_multiply(rtdm_ctx *c, rtdm_mat Cm, rtdm_mat Am, rtdm_mat Bm, int op_a, int op_b, double alr,
                  double ali, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    multiply(c, Cm, Am, Bm, op_a, op_b, alr, ali, (hipStream_t)stream, nullptr, 0);
    API_END(c)
}

int rtdm_multiply_noalloc(rtdm_ctx *c, rtdm_mat Cm, rtdm_mat Am, rtdm_mat Bm, int op_a, int op_b, double alr,
                          double ali, void *stream)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    multiply(c, Cm, Am, Bm, op_a, op_b, alr, ali, (hipStream_t)stream, static_scratch(c->device),
             kStaticScratchBytes);
    API_END(c)
}

int rtdm_schedule_stats(rtdm_ctx *c, rtdm_prod prod, int64_t *outputs, int64_t *triples)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    require(c->ranges_set, "set_ranges first");
    RT_CHECK(prod >= 0 && prod < RTDM_PROD_COUNT, RTDM_E_ARG, "bad product kind");
    Sched &S = schedule(c, prod);
    if (outputs) *outputs = S.nout;
    if (triples) *triples = S.ntrip;
    API_END(c)
}

int rtdm_timing(rtdm_ctx *c, int enable)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_HIP(hipDeviceSynchronize());
    c->recs.clear();
    c->timing = enable != 0;
    API_END(c)
}

int rtdm_timing_stats(rtdm_ctx *c, rtdm_prod prod, int64_t *launches, double *total_ms, double *flops)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    RT_CHECK(prod >= 0 && prod < RTDM_PROD_COUNT, RTDM_E_ARG, "bad product kind");
    RT_HIP(hipDeviceSynchronize());
    int64_t n = 0;
    double ms = 0.0, fl = 0.0;
    for (const auto &r : c->recs) {
        if (r.prod != prod) continue;
        float t = 0.0f;
        RT_HIP(hipEventElapsedTime(&t, c->events[r.ev], c->events[r.ev + 1]));
        ++n;
        ms += t;
        fl += r.flops;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (flops) *flops = fl;
    API_END(c)
}

int rtdm_inverse_info(rtdm_ctx *c, int *iters_total, int *fell_back)
{
    if (!c) return RTDM_E_ARG;
    if (iters_total) *iters_total = c->inv_iters_total;
    if (fell_back) *fell_back = c->inv_fell_back;
    c->err.clear();
    return RTDM_OK;
}

int rtdm_mlp_params(rtdm_ctx *c, int64_t *n_params, int *in, int *hidden, int *out)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    if (n_params) *n_params = c->mlp.np;
    if (in) *in = c->mlp.in;
    if (hidden) *hidden = kMlpHidden;
    if (out) *out = c->mlp.out;
    API_END(c)
}

int rtdm_mlp_set_weights(rtdm_ctx *c, const float *w, int64_t n)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    MlpState &M = c->mlp;
    RT_CHECK(w && n == M.np, RTDM_E_ARG, "weight count does not match the network");
    for (int64_t e = 0; e < n; ++e) RT_CHECK(std::isfinite(w[e]), RTDM_E_NUMERIC, "non-finite weight");
    RT_HIP(hipMemcpy(M.w.p, w, M.w.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemset(M.m.p, 0, M.m.bytes()));
    RT_HIP(hipMemset(M.v.p, 0, M.v.bytes()));
    M.step = 0;
    mlp_sync_half(c, nullptr);
    RT_HIP(hipDeviceSynchronize());
    M.ready = true;
    API_END(c)
}

int rtdm_mlp_get_weights(rtdm_ctx *c, float *w, int64_t n)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    RT_CHECK(w && n == c->mlp.np, RTDM_E_ARG, "weight count does not match the network");
    RT_HIP(hipMemcpy(w, c->mlp.w.p, c->mlp.w.bytes(), hipMemcpyDeviceToHost));
    API_END(c)
}

int rtdm_mlp_init(rtdm_ctx *c, uint64_t seed)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    MlpState &M = c->mlp;
    std::vector<float> w(M.np, 0.0f);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const double a1 = 1.0 / std::sqrt((double)M.in), a2 = 0.1 / std::sqrt((double)kMlpHidden);
    for (int64_t e = 0; e < M.nw1; ++e) w[e] = (float)(a1 * U(rng));
    for (int64_t e = 0; e < M.nw2; ++e) w[M.nw1 + M.nb1 + e] = (float)(a2 * U(rng));
    RT_HIP(hipMemcpy(M.w.p, w.data(), M.w.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemset(M.m.p, 0, M.m.bytes()));
    RT_HIP(hipMemset(M.v.p, 0, M.v.bytes()));
    M.step = 0;
    mlp_sync_half(c, nullptr);
    RT_HIP(hipDeviceSynchronize());
    M.ready = true;
    API_END(c)
}

int rtdm_mlp_collect(rtdm_ctx *c, int64_t max_samples, uint64_t seed, int64_t *total)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    RT_CHECK(!c->mixed, RTDM_E_UNSUPPORTED, "training samples need equal block sizes");
    set_device(c);
    require(c->ranges_set && c->uploaded[RTDM_MAT_S] && c->X_valid, "build the inverse first");
    RT_CHECK(max_samples >= 0, RTDM_E_ARG, "max_samples < 0");
    mlp_configure(c);
    MlpState &M = c->mlp;
    const Pattern &ps = pat_of(c, R_HS);
    std::vector<int32_t> pos(ps.nnzb);
    std::iota(pos.begin(), pos.end(), 0);
    std::mt19937_64 rng(seed);
    for (int64_t e = (int64_t)pos.size() - 1; e > 0; --e) {
        std::uniform_int_distribution<int64_t> pick(0, e);
        std::swap(pos[e], pos[pick(rng)]);
    }
    const int64_t k = std::min<int64_t>(max_samples, (int64_t)pos.size());
    pos.resize(k);
    std::sort(pos.begin(), pos.end());
    std::vector<int32_t> hs2p(ps.nnzb);
    RT_HIP(hipMemcpy(hs2p.data(), c->hs_to_p.p, c->hs_to_p.bytes(), hipMemcpyDeviceToHost));
    std::vector<int32_t> xo(k);
    for (int64_t e = 0; e < k; ++e) xo[e] = hs2p[pos[e]];
    if (M.ns + k > M.cap) {
        const int64_t cap = std::max<int64_t>(M.ns + k, 2 * M.cap);
        DBuf<float> nx, nt;
        nx.alloc((size_t)cap * M.in);
        nt.alloc((size_t)cap * M.out);
        if (M.ns > 0) {
            RT_HIP(hipMemcpy(nx.p, M.ds_x.p, (size_t)M.ns * M.in * sizeof(float), hipMemcpyDeviceToDevice));
            RT_HIP(hipMemcpy(nt.p, M.ds_t.p, (size_t)M.ns * M.out * sizeof(float), hipMemcpyDeviceToDevice));
        }
        M.ds_x = std::move(nx);
        M.ds_t = std::move(nt);
        M.cap = cap;
    }
    DBuf<int32_t> blk, xof;
    blk.alloc(std::max<int64_t>(k, 1));
    xof.alloc(std::max<int64_t>(k, 1));
    if (k > 0) {
        RT_HIP(hipMemcpy(blk.p, pos.data(), k * sizeof(int32_t), hipMemcpyHostToDevice));
        RT_HIP(hipMemcpy(xof.p, xo.data(), k * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    const double inv_r = c->radius[R_HS] > 0 ? 1.0 / c->radius[R_HS] : 1.0;
    launch_mlp_desc(nullptr, k, c->b, blk.p, ps.d_rowof.p, ps.d_col.p, c->d_xyz.p, c->mats[RTDM_MAT_S].re.p,
                    inv_r, M.ds_x.p + (size_t)M.ns * M.in);
    launch_mlp_target(nullptr, k, c->b, blk.p, xof.p, ps.d_rowof.p, ps.d_col.p, c->mats[RTDM_MAT_S].re.p,
                      c->mats[RTDM_MAT_X].re.p, M.ds_t.p + (size_t)M.ns * M.out);
    RT_HIP(hipDeviceSynchronize());
    M.ns += k;
    if (total) *total = M.ns;
    API_END(c)
}

int rtdm_mlp_clear(rtdm_ctx *c)
{
    if (!c) return RTDM_E_ARG;
    c->mlp.ns = 0;
    c->err.clear();
    return RTDM_OK;
}

int rtdm_mlp_train(rtdm_ctx *c, int epochs, int batch, double lr, uint64_t seed, double *loss)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    MlpState &M = c->mlp;
    require(M.ready && M.ns > 0, "initialise the network and collect samples first");
    RT_CHECK(epochs >= 1 && batch >= 1 && lr > 0 && std::isfinite(lr), RTDM_E_ARG, "bad training arguments");
    const int64_t bs = std::min<int64_t>(batch, M.ns);
    mlp_work(c, bs);
    M.idx.alloc(M.ns);
    std::vector<int32_t> perm(M.ns);
    double last = 0.0;
    for (int ep = 0; ep < epochs; ++ep) {
        std::iota(perm.begin(), perm.end(), 0);
        std::mt19937_64 rng(seed + 7919ull * (uint64_t)ep);
        for (int64_t e = (int64_t)perm.size() - 1; e > 0; --e) {
            std::uniform_int_distribution<int64_t> pick(0, e);
            std::swap(perm[e], perm[pick(rng)]);
        }
        RT_HIP(hipMemcpy(M.idx.p, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        double sum = 0.0;
        int64_t cnt = 0;
        for (int64_t b0 = 0; b0 + bs <= M.ns; b0 += bs) {
            const double l = mlp_loss_grad(c, bs, M.idx.p + b0, M.ds_x.p, M.ds_t.p, nullptr);
            launch_adam(nullptr, M.np, M.nw1, M.nb1, M.nw2, M.grad.p, M.w.p, M.m.p, M.v.p, (float)lr, 0.9,
                        0.999, 1e-8f, ++M.step, M.w1h.p, M.w2h.p);
            sum += l * bs;
            cnt += bs;
        }
        last = sum / (double)cnt;
        RT_CHECK(std::isfinite(last), RTDM_E_NUMERIC, "training loss is not finite");
    }
    RT_HIP(hipDeviceSynchronize());
    if (loss) *loss = last;
    API_END(c)
}

int rtdm_mlp_loss_grad(rtdm_ctx *c, int64_t n, const float *desc, const float *target, double *loss, float *grad)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    MlpState &M = c->mlp;
    require(M.ready, "initialise the network first");
    RT_CHECK(n >= 1 && desc && target, RTDM_E_ARG, "bad samples");
    M.tx.alloc((size_t)n * M.in);
    M.tt.alloc((size_t)n * M.out);
    RT_HIP(hipMemcpy(M.tx.p, desc, M.tx.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(M.tt.p, target, M.tt.bytes(), hipMemcpyHostToDevice));
    const double l = mlp_loss_grad(c, n, nullptr, M.tx.p, M.tt.p, nullptr);
    if (loss) *loss = l;
    if (grad) RT_HIP(hipMemcpy(grad, M.grad.p, M.grad.bytes(), hipMemcpyDeviceToHost));
    API_END(c)
}

int rtdm_mlp_step(rtdm_ctx *c, int64_t n, const float *desc, const float *target, double lr, double *loss)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    MlpState &M = c->mlp;
    require(M.ready, "initialise the network first");
    RT_CHECK(n >= 1 && desc && target && lr > 0 && std::isfinite(lr), RTDM_E_ARG, "bad samples or learning rate");
    M.tx.alloc((size_t)n * M.in);
    M.tt.alloc((size_t)n * M.out);
    RT_HIP(hipMemcpy(M.tx.p, desc, M.tx.bytes(), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(M.tt.p, target, M.tt.bytes(), hipMemcpyHostToDevice));
    const double l = mlp_loss_grad(c, n, nullptr, M.tx.p, M.tt.p, nullptr);
    launch_adam(nullptr, M.np, M.nw1, M.nb1, M.nw2, M.grad.p, M.w.p, M.m.p, M.v.p, (float)lr, 0.9, 0.999, 1e-8f,
                ++M.step, M.w1h.p, M.w2h.p);
    RT_HIP(hipDeviceSynchronize());
    if (loss) *loss = l;
    API_END(c)
}

int rtdm_mlp_predict(rtdm_ctx *c, int64_t n, const float *desc, float *y)
{
    if (!c) return RTDM_E_ARG;
    API_BEGIN
    set_device(c);
    mlp_configure(c);
    MlpState &M = c->mlp;
    require(M.ready, "initialise the network first");
    RT_CHECK(n >= 1 && desc && y, RTDM_E_ARG, "bad samples");
    M.tx.alloc((size_t)n * M.in);
    mlp_work(c, n);
    RT_HIP(hipMemcpy(M.tx.p, desc, M.tx.bytes(), hipMemcpyHostToDevice));
    launch_mlp_forward(nullptr, n, M.in, M.out, nullptr, M.tx.p, M.w1h.p, mlp_b1(M), M.w2h.p, mlp_b2(M), nullptr,
                       M.y.p);
    RT_HIP(hipMemcpy(y, M.y.p, (size_t)n * M.out * sizeof(float), hipMemcpyDeviceToHost));
    API_END(c)
}

const char *rtdm_last_error(const rtdm_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

}  // extern "C"

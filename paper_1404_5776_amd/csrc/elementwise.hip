// Block-wise and reduction kernels around the truncated products: Taylor-sum
// updates, Hermitisation, the kick, Mulliken charges, the on-site H model,
// observables and the block-Jacobi start of the inverse iteration.
//
// Every reduction is deterministic: a fixed grid of kRedBlocks workgroups,
// each thread summing a fixed strided subset in a fixed order, a fixed LDS
// tree per workgroup, then one workgroup summing the partials in a fixed
// tree.  Results are therefore bit-identical from run to run.
#include <cmath>

#include "internal.h"

namespace rtdm {

constexpr int kT = 256;

// ----------------------------------------------------------------- helpers

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-tree reduction of 4 slots (0..2 sums, 3 max) over a workgroup of kT threads.
__device__ inline void block_reduce4(double v[4], double *sh)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k * kT + t] = v[k];
    __syncthreads();
    for (int w = kT / 2; w >= 1; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sh[k * kT + t] += sh[k * kT + t + w];
            sh[3 * kT + t] = fmax(sh[3 * kT + t], sh[3 * kT + t + w]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = sh[k * kT];
}

__device__ inline void write_partials(double v[4], double *partials)
{
    __shared__ double sh[4 * kT];
    block_reduce4(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) partials[blockIdx.x * 4 + k] = v[k];
    }
}

// ----------------------------------------------------------------- elementwise

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double c,
                        const double *__restrict__ y, double *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = y ? a * x[e] + c * y[e] : a * x[e];
}

void launch_axpby(hipStream_t s, int64_t n, double a, const double *x, double c, const double *y,
                  double *out)
{
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)g), dim3(kT), 0, s, n, a, x, c, y, out);
    RT_HIP(hipGetLastError());
}

__global__ void k_add_identity(int64_t n_atoms, int b, const int32_t *__restrict__ diag, double val,
                               double *__restrict__ m)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_atoms * b) return;
    const int64_t i = e / b;
    const int a = (int)(e % b);
    m[(int64_t)diag[i] * b * b + a * b + a] += val;
}

void launch_add_identity(hipStream_t s, int64_t n_atoms, int b, const int32_t *diag, double val,
                         double *m)
{
    const int64_t n = n_atoms * b;
    if (n == 0) return;
    hipLaunchKernelGGL(k_add_identity, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, n_atoms,
                       b, diag, val, m);
    RT_HIP(hipGetLastError());
}

__global__ void k_kick(int64_t nnzb, int b, const int32_t *__restrict__ rowof,
                       const int32_t *__restrict__ col, const double *__restrict__ xyz, double kx,
                       double ky, double kz, double *__restrict__ kr, double *__restrict__ ki)
{
    const int bb = b * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzb * bb;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / bb;
        const int i = rowof[p], j = col[p];
        const double ph = kx * (xyz[3 * i] - xyz[3 * j]) + ky * (xyz[3 * i + 1] - xyz[3 * j + 1]) +
                          kz * (xyz[3 * i + 2] - xyz[3 * j + 2]);
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double xr = kr[e], xi = ki[e];
        kr[e] = cs * xr - sn * xi;
        ki[e] = cs * xi + sn * xr;
    }
}

void launch_kick(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof, const int32_t *col,
                 const double *xyz, double kx, double ky, double kz, double *kr, double *ki)
{
    const int64_t n = nnzb * b * b;
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_kick, dim3((unsigned)g), dim3(kT), 0, s, nnzb, b, rowof, col, xyz, kx, ky,
                       kz, kr, ki);
    RT_HIP(hipGetLastError());
}

// K_ij[a][c] = (Kn_ij[a][c] + conj(Kn_ji[c][a])) / 2
__global__ __launch_bounds__(kT) void k_hermitize(int64_t nnzb, int b,
                                                  const int32_t *__restrict__ trans,
                                                  const double *__restrict__ knr,
                                                  const double *__restrict__ kni,
                                                  double *__restrict__ kr, double *__restrict__ ki,
                                                  double *__restrict__ partials)
{
    const int bb = b * b;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nnzb * bb;
         e += (int64_t)kRedBlocks * kT) {
        const int64_t p = e / bb;
        const int w = (int)(e - p * bb);
        const int a = w / b, c = w - a * b;
        const int64_t pe = (int64_t)trans[p] * bb + c * b + a;
        const double xr = knr[e], xi = kni[e], yr = knr[pe], yi = -kni[pe];
        kr[e] = 0.5 * (xr + yr);
        ki[e] = 0.5 * (xi + yi);
        const double dr = xr - yr, di = xi - yi;
        v[0] += dr * dr + di * di;
        v[1] += xr * xr + xi * xi;
    }
    write_partials(v, partials);
}

void launch_hermitize(hipStream_t s, int64_t nnzb, int b, const int32_t *trans, const double *knr,
                      const double *kni, double *kr, double *ki, double *partials)
{
    hipLaunchKernelGGL(k_hermitize, dim3(kRedBlocks), dim3(kT), 0, s, nnzb, b, trans, knr, kni, kr,
                       ki, partials);
    RT_HIP(hipGetLastError());
}

// One wave per atom: q_i = Re sum_{j in S row i, (i,j) in K} sum_{a,c} K_ij[a][c] S_ji[c][a]
__global__ __launch_bounds__(kT) void k_mulliken(int64_t n_atoms, int b,
                                                 const int64_t *__restrict__ s_ptr,
                                                 const int32_t *__restrict__ s_trans,
                                                 const int32_t *__restrict__ s_to_k,
                                                 const double *__restrict__ sv,
                                                 const double *__restrict__ kr,
                                                 double *__restrict__ q)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (i >= n_atoms) return;
    const int bb = b * b;
    // the row's (block, element) pairs flattened, 64 per pass, so every lane
    // works and a pass has 64 independent loads (b = 4: four blocks at once)
    const int64_t p0 = s_ptr[i];
    const int64_t nel = (s_ptr[i + 1] - p0) * bb;
    double acc = 0.0;
    for (int64_t x = lane; x < nel; x += 64) {
        const int64_t p = p0 + x / bb;
        const int w = (int)(x % bb);
        const int kb = s_to_k[p];
        if (kb < 0) continue;
        const int a = w / b, c = w - a * b;
        acc += kr[(int64_t)kb * bb + w] * sv[(int64_t)s_trans[p] * bb + c * b + a];
    }
    acc = wave_sum(acc);
    if (lane == 0) q[i] = acc;
}

void launch_mulliken(hipStream_t s, int64_t n_atoms, int b, const int64_t *s_ptr,
                     const int32_t *s_trans, const int32_t *s_to_k, const double *sv,
                     const double *kr, double *q)
{
    if (n_atoms == 0) return;
    const int per = kT / 64;
    hipLaunchKernelGGL(k_mulliken, dim3((unsigned)((n_atoms + per - 1) / per)), dim3(kT), 0, s,
                       n_atoms, b, s_ptr, s_trans, s_to_k, sv, kr, q);
    RT_HIP(hipGetLastError());
}

// H_ii += g (q_eff,i - q_ref,i) on the diagonal of atom i's block, with the
// charges at the step's time point q_eff = q_a + theta (q_x - q_y):
// extrapolation (q_x, q_y) = (q(t), q(t - dt)) or interpolation
// (q(t + dt), q(t)), q_a = q(t).
__global__ void k_onsite_shift(int64_t n_atoms, int b, const int32_t *__restrict__ diag,
                               const int32_t *__restrict__ nbf, double gain, const double *__restrict__ q_a,
                               double theta, const double *__restrict__ q_x, const double *__restrict__ q_y,
                               const double *__restrict__ q_ref, double *__restrict__ h)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_atoms * b) return;
    const int64_t i = e / b;
    const int a = (int)(e % b);
    if (nbf && a >= nbf[i]) return;            // a padded function of a smaller atom
    const double q = q_a[i] + theta * (q_x[i] - q_y[i]);
    h[(int64_t)diag[i] * b * b + a * b + a] += gain * (q - q_ref[i]);
}

// A = A0 + X D on the range of X and A, with A0 = P(X H0) and D the on-site
// term of the Mulliken model: D_jj = g (q_a + theta (q_x - q_y) - q_ref)_j on
// each of atom j's own functions.  Since D only scales block columns of X,
// P(X (H0 + D)) = P(X H0) + X D exactly in arithmetic; the sums are rounded
// differently from the product of X with H0 + D.
template <typename I>
__global__ void k_a_onsite(I n, int b, const int32_t *__restrict__ col, const int32_t *__restrict__ nbf,
                           double gain, const double *__restrict__ q_a, double theta,
                           const double *__restrict__ q_x, const double *__restrict__ q_y,
                           const double *__restrict__ q_ref, const double *__restrict__ a0,
                           const double *__restrict__ x, double *__restrict__ a)
{
    const I bb = (I)b * b;
    for (I e = (I)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (I)gridDim.x * blockDim.x) {
        const I p = e / bb;
        const int cc = (int)((e - p * bb) % (I)b);
        const int j = col[p];
        double v = a0[e];
        if (!nbf || cc < nbf[j]) {
            const double q = q_a[j] + theta * (q_x[j] - q_y[j]);
            v += x[e] * (gain * (q - q_ref[j]));
        }
        a[e] = v;
    }
}

void launch_a_onsite(hipStream_t s, int64_t nnzb, int b, const int32_t *col, const int32_t *nbf, double gain,
                     const double *q_a, double theta, const double *q_x, const double *q_y, const double *q_ref,
                     const double *a0, const double *x, double *a)
{
    const int64_t n = nnzb * b * b;
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    // 32-bit index arithmetic (the divisions by b^2 and b) whenever it fits
    if (n + (int64_t)g * kT < ((int64_t)1 << 32))
        hipLaunchKernelGGL(k_a_onsite<uint32_t>, dim3((unsigned)g), dim3(kT), 0, s, (uint32_t)n, b, col, nbf, gain,
                           q_a, theta, q_x, q_y, q_ref, a0, x, a);
    else
        hipLaunchKernelGGL(k_a_onsite<int64_t>, dim3((unsigned)g), dim3(kT), 0, s, n, b, col, nbf, gain, q_a, theta,
                           q_x, q_y, q_ref, a0, x, a);
    RT_HIP(hipGetLastError());
}

void launch_onsite_shift(hipStream_t s, int64_t n_atoms, int b, const int32_t *diag, const int32_t *nbf, double gain,
                         const double *q_a, double theta, const double *q_x, const double *q_y,
                         const double *q_ref, double *h)
{
    const int64_t n = n_atoms * b;
    if (n == 0) return;
    hipLaunchKernelGGL(k_onsite_shift, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, n_atoms,
                       b, diag, nbf, gain, q_a, theta, q_x, q_y, q_ref, h);
    RT_HIP(hipGetLastError());
}

// H_ij += (E(t) . ((r_i + r_j)/2 - r_c)) S_ij on the pattern of S, with the
// Gaussian profile E(t) = E0 exp(-(t - t0)^2 / (2 sigma^2)) at the device
// step time t = tt[0] + (st[1] + theta) tt[1] and r_c the centre of the
// group of atom i (centre[3 g..3 g+2]).
__global__ void k_field(int64_t nnzb, int b, const int32_t *__restrict__ rowof,
                        const int32_t *__restrict__ col, const double *__restrict__ xyz,
                        const int32_t *__restrict__ group, const double *__restrict__ centre,
                        const double *__restrict__ sv, double ex, double ey, double ez, double t0,
                        double sigma, const int64_t *__restrict__ st, const double *__restrict__ tt,
                        double theta, double *__restrict__ h)
{
    const int64_t bb = (int64_t)b * b;
    const double t = tt[0] + ((double)st[1] + theta) * tt[1];
    const double d = t - t0;
    const double f = exp(-(d * d) / (2.0 * sigma * sigma));
    const double E[3] = {ex * f, ey * f, ez * f};
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzb * bb;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / bb;
        const int64_t i = rowof[p], j = col[p];
        const double *c = centre + 3 * (group ? group[i] : 0);
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) v += 0.5 * ((xyz[3 * i + k] - c[k]) + (xyz[3 * j + k] - c[k])) * E[k];
        h[e] += v * sv[e];
    }
}

void launch_field(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof, const int32_t *col,
                  const double *xyz, const int32_t *group, const double *centre, const double *sv,
                  const double E0[3], double t0, double sigma, const int64_t *st, const double *tt,
                  double theta, double *h)
{
    const int64_t n = nnzb * (int64_t)b * b;
    if (n == 0) return;
    const int64_t g = std::min<int64_t>((n + kT - 1) / kT, 65536);
    hipLaunchKernelGGL(k_field, dim3((unsigned)g), dim3(kT), 0, s, nnzb, b, rowof, col, xyz, group, centre,
                       sv, E0[0], E0[1], E0[2], t0, sigma, st, tt, theta, h);
    RT_HIP(hipGetLastError());
}

// Damped transform of a dipole trace, one thread per frequency, the sum over
// time points in order: F[f](w) = sum_{k=0}^{n} f(t_k) exp((i w - gamma) t_k) dt,
// t_k = k dt, f = P - P0 (zero at k = 0; P(t_k) = trace[(k-1) * stride + off
// + 0..2] for k >= 1).  The field transform is -kappa (kick) or the sum over
// the Gaussian field sampled at t_k.  alpha[w][j] = F[P_j - P0_j] / F[E_j]
// (NaN where F[E_j] = 0), strength[w] = (2 w / pi) Im(sum_j alpha_jj / 3).
__global__ void k_spectrum(int64_t n_omega, const double *__restrict__ omega, double gamma, double dt,
                           int64_t n, const double *__restrict__ trace, int64_t stride, int64_t off,
                           double p0x, double p0y, double p0z, int kick, double kx, double ky, double kz,
                           double t0, double sigma, double *__restrict__ alpha, double *__restrict__ strength)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_omega) return;
    const double om = omega[w];
    const double P0[3] = {p0x, p0y, p0z};
    const double E0[3] = {kx, ky, kz};
    double fr[3] = {0.0, 0.0, 0.0}, fi[3] = {0.0, 0.0, 0.0};
    double er[3] = {0.0, 0.0, 0.0}, ei[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k <= n; ++k) {
        const double t = (double)k * dt;
        const double m = exp(-gamma * t) * dt;
        double sn, cs;
        sincos(om * t, &sn, &cs);
        const double pr = m * cs, pi = m * sn;
        if (k > 0) {
            const double *row = trace + (k - 1) * stride + off;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double f = row[j] - P0[j];
                fr[j] += pr * f;
                fi[j] += pi * f;
            }
        }
        if (!kick) {
            const double d = t - t0;
            const double g = exp(-(d * d) / (2.0 * sigma * sigma));
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                er[j] += pr * (E0[j] * g);
                ei[j] += pi * (E0[j] * g);
            }
        }
    }
    double tr_im = 0.0;
    for (int j = 0; j < 3; ++j) {
        double ar, ai;
        if (kick) {
            er[j] = -E0[j];
            ei[j] = 0.0;
        }
        if (er[j] == 0.0 && ei[j] == 0.0) {
            ar = ai = __builtin_nan("");
        } else {
            const double den = er[j] * er[j] + ei[j] * ei[j];
            ar = (fr[j] * er[j] + fi[j] * ei[j]) / den;
            ai = (fi[j] * er[j] - fr[j] * ei[j]) / den;
            tr_im += ai;
        }
        alpha[(w * 3 + j) * 2] = ar;
        alpha[(w * 3 + j) * 2 + 1] = ai;
    }
    if (strength) strength[w] = 2.0 * om / M_PI * (tr_im / 3.0);
}

void launch_spectrum(hipStream_t s, int64_t n_omega, const double *omega, double gamma, double dt, int64_t n,
                     const double *trace, int64_t stride, int64_t off, const double P0[3], int kick,
                     const double E0[3], double t0, double sigma, double *alpha, double *strength)
{
    if (n_omega == 0) return;
    hipLaunchKernelGGL(k_spectrum, dim3((unsigned)((n_omega + 63) / 64)), dim3(64), 0, s, n_omega, omega, gamma,
                       dt, n, trace, stride, off, P0[0], P0[1], P0[2], kick, E0[0], E0[1], E0[2], t0, sigma,
                       alpha, strength);
    RT_HIP(hipGetLastError());
}

// Single workgroup: centroid, dipole P = -sum (r_i - r_c) q_i, Tr(KS) = sum q_i.
// With a step state st/tt the row is out + 8 * st[0], the time tt[0] +
// (st[1] + 1) * tt[1] (k_step_end advances both counters); without one (st null) the
// row is `out` and the time `t`.
__global__ __launch_bounds__(kT) void k_observables(int64_t n, const double *__restrict__ xyz,
                                                    const double *__restrict__ centre,
                                                    const double *__restrict__ q,
                                                    const double *__restrict__ herm_sums, double t,
                                                    double *__restrict__ out, int64_t *st,
                                                    const double *__restrict__ tt)
{
    __shared__ double sh[4 * kT];
    const double cx = centre[0], cy = centre[1], cz = centre[2];
    double w[4] = {0.0, 0.0, 0.0, 0.0};
    double tr = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kT) {
        const double qi = q[i];
        w[0] -= (xyz[3 * i] - cx) * qi;
        w[1] -= (xyz[3 * i + 1] - cy) * qi;
        w[2] -= (xyz[3 * i + 2] - cz) * qi;
        tr += qi;
    }
    w[3] = 0.0;
    block_reduce4(w, sh);
    __syncthreads();
    double u[4] = {tr, 0.0, 0.0, 0.0};
    block_reduce4(u, sh);
    if (threadIdx.x == 0) {
        double *row = st ? out + 8 * st[0] : out;
        row[0] = st ? tt[0] + (double)(st[1] + 1) * tt[1] : t;
        row[1] = w[0];
        row[2] = w[1];
        row[3] = w[2];
        row[4] = u[0];
        row[5] = herm_sums ? (herm_sums[1] > 0.0 ? sqrt(herm_sums[0] / herm_sums[1]) : 0.0) : 0.0;
        row[6] = __builtin_nan("");
        row[7] = 0.0;
    }
}

void launch_observables(hipStream_t s, int64_t n_atoms, const double *xyz, const double *centre, const double *q,
                        const double *herm_sums, double t, double *row)
{
    hipLaunchKernelGGL(k_observables, dim3(1), dim3(kT), 0, s, n_atoms, xyz, centre, q, herm_sums, t, row,
                       (int64_t *)nullptr, (const double *)nullptr);
    RT_HIP(hipGetLastError());
}

// Advance the step state after a step's observables (st[0]++, st[1]++).
__global__ void k_step_end(int64_t *st)
{
    if (threadIdx.x == 0) {
        st[0] += 1;
        st[1] += 1;
    }
}

void launch_observables_step(hipStream_t s, int64_t n_atoms, const double *xyz, const double *centre,
                             const double *q, const double *herm_sums, double *obs, int64_t *st, const double *tt)
{
    hipLaunchKernelGGL(k_observables, dim3(1), dim3(kT), 0, s, n_atoms, xyz, centre, q, herm_sums, 0.0, obs, st,
                       tt);
    RT_HIP(hipGetLastError());
}

void launch_step_end(hipStream_t s, int64_t *st)
{
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, s, st);
    RT_HIP(hipGetLastError());
}

// One thread per atom: Gauss-Jordan with partial pivoting on [S_ii | I] in scratch.
__global__ void k_block_inverse(int64_t n_atoms, int b, const int32_t *__restrict__ s_diag,
                                const double *__restrict__ sv, const int32_t *__restrict__ x_diag,
                                double *__restrict__ xv, double *__restrict__ scratch)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_atoms) return;
    const int w = 2 * b;
    double *m = scratch + i * (int64_t)b * w;
    const double *src = sv + (int64_t)s_diag[i] * b * b;
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < w; ++c) m[r * w + c] = c < b ? src[r * b + c] : (c - b == r ? 1.0 : 0.0);
    for (int col = 0; col < b; ++col) {
        int piv = col;
        double best = fabs(m[col * w + col]);
        for (int r = col + 1; r < b; ++r)
            if (fabs(m[r * w + col]) > best) { best = fabs(m[r * w + col]); piv = r; }
        if (piv != col)
            for (int c = 0; c < w; ++c) {
                const double tmp = m[col * w + c];
                m[col * w + c] = m[piv * w + c];
                m[piv * w + c] = tmp;
            }
        const double inv = 1.0 / m[col * w + col];
        for (int c = 0; c < w; ++c) m[col * w + c] *= inv;
        for (int r = 0; r < b; ++r) {
            if (r == col) continue;
            const double f = m[r * w + col];
            if (f != 0.0)
                for (int c = 0; c < w; ++c) m[r * w + c] -= f * m[col * w + c];
        }
    }
    double *dst = xv + (int64_t)x_diag[i] * b * b;
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) dst[r * b + c] = m[r * w + b + c];
}

void launch_block_inverse(hipStream_t s, int64_t n_atoms, int b, const int32_t *s_diag,
                          const double *sv, const int32_t *x_diag, double *xv, double *scratch)
{
    if (n_atoms == 0) return;
    hipLaunchKernelGGL(k_block_inverse, dim3((unsigned)((n_atoms + 63) / 64)), dim3(64), 0, s,
                       n_atoms, b, s_diag, sv, x_diag, xv, scratch);
    RT_HIP(hipGetLastError());
}

__global__ void k_row_abs_max(int64_t n_atoms, int b, const int64_t *__restrict__ s_ptr,
                              const double *__restrict__ sv, double *__restrict__ atom_max)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_atoms) return;
    double best = 0.0;
    for (int a = 0; a < b; ++a) {
        double sum = 0.0;
        for (int64_t p = s_ptr[i]; p < s_ptr[i + 1]; ++p)
            for (int c = 0; c < b; ++c) sum += fabs(sv[p * b * b + a * b + c]);
        best = fmax(best, sum);
    }
    atom_max[i] = best;
}

void launch_row_abs_max(hipStream_t s, int64_t n_atoms, int b, const int64_t *s_ptr,
                        const double *sv, double *atom_max)
{
    if (n_atoms == 0) return;
    hipLaunchKernelGGL(k_row_abs_max, dim3((unsigned)((n_atoms + kT - 1) / kT)), dim3(kT), 0, s,
                       n_atoms, b, s_ptr, sv, atom_max);
    RT_HIP(hipGetLastError());
}

__global__ void k_transpose_blocks(int64_t nblocks, int b, const double *__restrict__ in,
                                   double *__restrict__ out)
{
    const int bb = b * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nblocks * bb;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / bb;
        const int w = (int)(e - p * bb);
        const int r = w / b, c = w - r * b;
        out[p * bb + c * b + r] = in[e];
    }
}

void launch_transpose_blocks(hipStream_t s, int64_t nblocks, int b, const double *in, double *out)
{
    const int64_t n = nblocks * b * b;
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_transpose_blocks, dim3((unsigned)g), dim3(kT), 0, s, nblocks, b, in, out);
    RT_HIP(hipGetLastError());
}

// out_ji = in_ij^dagger for every block p = (i, j) of a pattern (trans[p] =
// the block (j, i)): out[trans[p]][c][r] = conj(in[p][r][c]).  B is the block
// size when fixed at compile time (4), else 0 and b is read at run time.
template <int B>
__global__ void k_conj_transpose(int64_t nnzb, int b, const int32_t *__restrict__ trans,
                                 const double *__restrict__ in_re, const double *__restrict__ in_im,
                                 double *__restrict__ out_re, double *__restrict__ out_im)
{
    const int bs = B ? B : b, bb = bs * bs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzb * bb;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / bb;
        const int w = (int)(e - p * bb);
        const int r = w / bs, c = w - r * bs;
        const int64_t o = (int64_t)trans[p] * bb + c * bs + r;
        out_re[o] = in_re[e];
        out_im[o] = -in_im[e];
    }
}

void launch_conj_transpose(hipStream_t s, int64_t nnzb, int b, const int32_t *trans, const double *in_re,
                           const double *in_im, double *out_re, double *out_im)
{
    const int64_t n = nnzb * b * b;
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    if (b == 4)
        hipLaunchKernelGGL(k_conj_transpose<4>, dim3((unsigned)g), dim3(kT), 0, s, nnzb, b, trans, in_re, in_im,
                           out_re, out_im);
    else
        hipLaunchKernelGGL(k_conj_transpose<0>, dim3((unsigned)g), dim3(kT), 0, s, nnzb, b, trans, in_re, in_im,
                           out_re, out_im);
    RT_HIP(hipGetLastError());
}

__global__ void k_to_f32(int64_t nblocks, int b, int transpose, const double *__restrict__ in,
                         float *__restrict__ out)
{
    const int bb = b * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nblocks * bb;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t o = e;
        if (transpose) {
            const int64_t p = e / bb;
            const int w = (int)(e - p * bb);
            const int r = w / b, c = w - r * b;
            o = p * bb + c * b + r;
        }
        out[o] = (float)in[e];
    }
}

void launch_to_f32(hipStream_t s, int64_t nblocks, int b, int transpose, const double *in, float *out)
{
    const int64_t n = nblocks * b * b;
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)g), dim3(kT), 0, s, nblocks, b, transpose, in, out);
    RT_HIP(hipGetLastError());
}

__global__ void k_axpy_f32(int64_t n, double a, const float *__restrict__ x, double *__restrict__ y)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        y[e] += a * (double)x[e];
}

void launch_axpy_f32(hipStream_t s, int64_t n, double a, const float *x, double *y)
{
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_axpy_f32, dim3((unsigned)g), dim3(kT), 0, s, n, a, x, y);
    RT_HIP(hipGetLastError());
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = v;
}

void launch_fill(hipStream_t s, int64_t n, double v, double *out)
{
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(kT), 0, s, n, v, out);
    RT_HIP(hipGetLastError());
}

// Step state kept on the device so that one captured step can be replayed:
// st[0] = next trace row, st[1] = steps done in this call, and
// tt[0] = time at the start of the call, tt[1] = dt.
__global__ void k_step_begin(int64_t *st, double *tt, double t0, double dt)
{
    if (threadIdx.x == 0) {
        st[1] = 0;
        tt[0] = t0;
        tt[1] = dt;
    }
}

void launch_step_begin(hipStream_t s, int64_t *st, double *tt, double t0, double dt)
{
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(64), 0, s, st, tt, t0, dt);
    RT_HIP(hipGetLastError());
}

// Per-group observables of the new K (one workgroup per group of contiguous
// atoms): centroid, dipole -sum (r_i - r_c) q_i and Tr(KS) = sum q_i, written
// to out[row][g][0..3] with row = st[0].
__global__ __launch_bounds__(kT) void k_group_obs(const int64_t *__restrict__ gptr,
                                                  const double *__restrict__ xyz,
                                                  const double *__restrict__ centre,
                                                  const double *__restrict__ q,
                                                  const int64_t *__restrict__ st, int64_t n_groups,
                                                  double *__restrict__ out)
{
    __shared__ double sh[4 * kT];
    const int64_t g = blockIdx.x;
    const int64_t a0 = gptr[g], a1 = gptr[g + 1];
    const double cx = centre[3 * g], cy = centre[3 * g + 1], cz = centre[3 * g + 2];
    double w[4] = {0.0, 0.0, 0.0, 0.0};
    double tr = 0.0;
    for (int64_t i = a0 + threadIdx.x; i < a1; i += kT) {
        const double qi = q[i];
        w[0] -= (xyz[3 * i] - cx) * qi;
        w[1] -= (xyz[3 * i + 1] - cy) * qi;
        w[2] -= (xyz[3 * i + 2] - cz) * qi;
        tr += qi;
    }
    block_reduce4(w, sh);
    __syncthreads();
    double u[4] = {tr, 0.0, 0.0, 0.0};
    block_reduce4(u, sh);
    if (threadIdx.x == 0) {
        double *o = out + (st[0] * n_groups + g) * 4;
        o[0] = w[0];
        o[1] = w[1];
        o[2] = w[2];
        o[3] = u[0];
    }
}

void launch_group_obs(hipStream_t s, int64_t n_groups, const int64_t *gptr, const double *xyz, const double *centre,
                      const double *q, const int64_t *st, double *out)
{
    if (n_groups == 0) return;
    hipLaunchKernelGGL(k_group_obs, dim3((unsigned)n_groups), dim3(kT), 0, s, gptr, xyz, centre, q, st, n_groups,
                       out);
    RT_HIP(hipGetLastError());
}

// K_ij *= exp(i kappa_g . (r_i - r_j)) with the kick of atom i's group (pairs
// never cross groups in a block-diagonal batch).
__global__ void k_kick_groups(int64_t nnzb, int b, const int32_t *__restrict__ rowof,
                              const int32_t *__restrict__ col, const double *__restrict__ xyz,
                              const int32_t *__restrict__ group, const double *__restrict__ kappa,
                              double *__restrict__ kr, double *__restrict__ ki)
{
    const int bb = b * b;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnzb * bb;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / bb;
        const int i = rowof[p], j = col[p];
        const double *k = kappa + 3 * group[i];
        const double ph = k[0] * (xyz[3 * i] - xyz[3 * j]) + k[1] * (xyz[3 * i + 1] - xyz[3 * j + 1]) +
                          k[2] * (xyz[3 * i + 2] - xyz[3 * j + 2]);
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double xr = kr[e], xi = ki[e];
        kr[e] = cs * xr - sn * xi;
        ki[e] = cs * xi + sn * xr;
    }
}

void launch_kick_groups(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof, const int32_t *col,
                        const double *xyz, const int32_t *group, const double *kappa, double *kr, double *ki)
{
    const int64_t n = nnzb * b * b;
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_kick_groups, dim3((unsigned)g), dim3(kT), 0, s, nnzb, b, rowof, col, xyz, group, kappa,
                       kr, ki);
    RT_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- reductions

__global__ __launch_bounds__(kT) void k_red_diff2(int64_t n, const double *__restrict__ x,
                                                  const double *__restrict__ y,
                                                  double *__restrict__ partials)
{
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)kRedBlocks * kT) {
        const double d = x[e] - y[e];
        v[0] += d * d;
        v[1] += x[e] * x[e];
        v[3] = fmax(v[3], fabs(d));
    }
    write_partials(v, partials);
}

void launch_red_diff2(hipStream_t s, int64_t n, const double *x, const double *y, double *partials)
{
    hipLaunchKernelGGL(k_red_diff2, dim3(kRedBlocks), dim3(kT), 0, s, n, x, y, partials);
    RT_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kT) void k_red_unitarity(int64_t nnzb_p, int b,
                                                      const int32_t *__restrict__ p_to_hs,
                                                      const double *__restrict__ sv,
                                                      const double *__restrict__ zr,
                                                      const double *__restrict__ zi,
                                                      double *__restrict__ partials)
{
    const int bb = b * b;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nnzb_p * bb;
         e += (int64_t)kRedBlocks * kT) {
        const int64_t p = e / bb;
        const int w = (int)(e - p * bb);
        const int hs = p_to_hs[p];
        const double sval = hs >= 0 ? sv[(int64_t)hs * bb + w] : 0.0;
        const double dr = zr[e] - sval, di = zi[e];
        const double m2 = dr * dr + di * di;
        const double m = sqrt(m2);
        v[0] += m2;
        v[1] += m;
        v[3] = fmax(v[3], m);
    }
    write_partials(v, partials);
}

void launch_red_unitarity(hipStream_t s, int64_t nnzb_p, int b, const int32_t *p_to_hs,
                          const double *sv, const double *zr, const double *zi, double *partials)
{
    hipLaunchKernelGGL(k_red_unitarity, dim3(kRedBlocks), dim3(kT), 0, s, nnzb_p, b, p_to_hs, sv, zr,
                       zi, partials);
    RT_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kT) void k_red_minus_identity(int64_t nnzb, int b,
                                                           const int32_t *__restrict__ rowof,
                                                           const int32_t *__restrict__ col,
                                                           const double *__restrict__ v,
                                                           double *__restrict__ partials)
{
    const int bb = b * b;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nnzb * bb;
         e += (int64_t)kRedBlocks * kT) {
        const int64_t p = e / bb;
        const int w = (int)(e - p * bb);
        const double id = (rowof[p] == col[p] && w % (b + 1) == 0) ? 1.0 : 0.0;
        const double d = v[e] - id;
        acc[0] += d * d;
        acc[1] += fabs(d);
        acc[3] = fmax(acc[3], fabs(d));
    }
    write_partials(acc, partials);
}

void launch_red_minus_identity(hipStream_t s, int64_t nnzb, int b, const int32_t *rowof,
                               const int32_t *col, const double *v, double *partials)
{
    hipLaunchKernelGGL(k_red_minus_identity, dim3(kRedBlocks), dim3(kT), 0, s, nnzb, b, rowof, col, v,
                       partials);
    RT_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kT) void k_red_sumsq(int64_t n, const double *__restrict__ x,
                                                  double *__restrict__ partials)
{
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)kRedBlocks * kT) {
        v[0] += x[e] * x[e];
        v[3] = fmax(v[3], fabs(x[e]));
    }
    write_partials(v, partials);
}

// Sum of the diagonal elements of the diagonal blocks (slot 0).
__global__ __launch_bounds__(kT) void k_red_trace(int64_t n_atoms, int b, const int32_t *__restrict__ diag,
                                                  const double *__restrict__ v, double *__restrict__ partials)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n_atoms * b; e += (int64_t)kRedBlocks * kT) {
        const int64_t i = e / b;
        const int a = (int)(e - i * b);
        acc[0] += v[(int64_t)diag[i] * b * b + a * (b + 1)];
    }
    write_partials(acc, partials);
}

void launch_red_trace(hipStream_t s, int64_t n_atoms, int b, const int32_t *diag, const double *v,
                      double *partials)
{
    hipLaunchKernelGGL(k_red_trace, dim3(kRedBlocks), dim3(kT), 0, s, n_atoms, b, diag, v, partials);
    RT_HIP(hipGetLastError());
}

// Gershgorin row discs of a block-sparse matrix: for element row (i, a),
// lohi = (c - r, c + r) with c = a_(ia,ia) and r = sum over the row's other
// elements of |a| (blocks of the row in order, each block's row summed first).
__global__ void k_gershgorin(int64_t n_atoms, int b, const int64_t *__restrict__ rowptr,
                             const int32_t *__restrict__ diag, const double *__restrict__ v,
                             double *__restrict__ lohi)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_atoms * b) return;
    const int64_t i = e / b;
    const int a = (int)(e - i * b);
    const int64_t bb = (int64_t)b * b;
    double rs = 0.0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        double t = 0.0;
        for (int c = 0; c < b; ++c) t += fabs(v[p * bb + a * b + c]);
        rs += t;
    }
    const double cen = v[(int64_t)diag[i] * bb + a * (b + 1)];
    const double rad = rs - fabs(cen);
    lohi[2 * e] = cen - rad;
    lohi[2 * e + 1] = cen + rad;
}

void launch_gershgorin(hipStream_t s, int64_t n_atoms, int b, const int64_t *rowptr, const int32_t *diag,
                       const double *v, double *lohi)
{
    const int64_t n = n_atoms * b;
    if (n == 0) return;
    hipLaunchKernelGGL(k_gershgorin, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, n_atoms, b, rowptr, diag,
                       v, lohi);
    RT_HIP(hipGetLastError());
}

void launch_red_sumsq(hipStream_t s, int64_t n, const double *x, double *partials)
{
    hipLaunchKernelGGL(k_red_sumsq, dim3(kRedBlocks), dim3(kT), 0, s, n, x, partials);
    RT_HIP(hipGetLastError());
}

void launch_red_max(hipStream_t s, int64_t n, const double *x, double *partials)
{
    launch_red_sumsq(s, n, x, partials);
}

// One workgroup of kT threads sums kRedBlocks partials (kRedBlocks = 2 kT).
__global__ __launch_bounds__(kT) void k_red_finish(const double *__restrict__ partials,
                                                   double *__restrict__ out)
{
    __shared__ double sh[4 * kT];
    const int t = threadIdx.x;
    double v[4];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = partials[t * 4 + k] + partials[(t + kT) * 4 + k];
    v[3] = fmax(partials[t * 4 + 3], partials[(t + kT) * 4 + 3]);
    block_reduce4(v, sh);
    if (t == 0)
        for (int k = 0; k < 4; ++k) out[k] = v[k];
}

void launch_red_finish(hipStream_t s, const double *partials, double *out)
{
    static_assert(kRedBlocks == 2 * kT, "finish kernel assumes two partials per thread");
    hipLaunchKernelGGL(k_red_finish, dim3(1), dim3(kT), 0, s, partials, out);
    RT_HIP(hipGetLastError());
}

__global__ void k_unit_to_row(const double *__restrict__ unit_sums,
                              const double *__restrict__ s_norm2, double *__restrict__ row)
{
    if (threadIdx.x == 0) row[6] = sqrt(unit_sums[0] / s_norm2[0]);
}

void launch_unit_to_row(hipStream_t s, const double *unit_sums, const double *s_norm2, double *row)
{
    hipLaunchKernelGGL(k_unit_to_row, dim3(1), dim3(64), 0, s, unit_sums, s_norm2, row);
    RT_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- layout

__global__ void k_split(int64_t n, const double *__restrict__ inter, double *__restrict__ re,
                        double *__restrict__ im)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        re[e] = inter[2 * e];
        if (im) im[e] = inter[2 * e + 1];
    }
}

void launch_split(hipStream_t s, int64_t n, const double *inter, double *re, double *im)
{
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_split, dim3((unsigned)g), dim3(kT), 0, s, n, inter, re, im);
    RT_HIP(hipGetLastError());
}

__global__ void k_interleave(int64_t n, const double *__restrict__ re, const double *__restrict__ im,
                             double *__restrict__ inter)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        inter[2 * e] = re[e];
        inter[2 * e + 1] = im ? im[e] : 0.0;
    }
}

void launch_interleave(hipStream_t s, int64_t n, const double *re, const double *im, double *inter)
{
    if (n == 0) return;
    int64_t g = (n + kT - 1) / kT;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_interleave, dim3((unsigned)g), dim3(kT), 0, s, n, re, im, inter);
    RT_HIP(hipGetLastError());
}

// x[0] += v (one thread): a device scalar corrected in stream order.
__global__ void k_add_scalar(double *x, double v)
{
    if (threadIdx.x == 0) x[0] += v;
}

void launch_add_scalar(hipStream_t s, double *x, double v)
{
    hipLaunchKernelGGL(k_add_scalar, dim3(1), dim3(64), 0, s, x, v);
    RT_HIP(hipGetLastError());
}

}  // namespace rtdm


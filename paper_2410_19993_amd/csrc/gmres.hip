// Krylov refinement of the condensed system (Sec. II.B's block-tridiagonal matrix A,
// one right-hand side V c per input vector): restarted flexible GMRES (Saad's FGMRES,
// right preconditioned) in float64 around the low-precision factor, after Carson and
// Higham's GMRES-based iterative refinement.  Each outer step forms the float64
// residual r = V c - A u, runs k Arnoldi steps on A M^-1 with M^-1 the float sweep
// of the factor (so an inexact, slightly varying preconditioner is allowed), solves
// the (k+1) x k least-squares problem, and adds the correction d = Z y to u.
//
// The kernels here are the batched vector operations of that loop over the panel
// layout of the refinement, [nslab][m][16][n_p] float64 (input vector b = 16 slab +
// col, row i, bit line j at ((slab m + i) 16 + col) n_p + j, zero for j >= n and for
// b >= B).  Reductions over a vector's m n_p entries run in a fixed order (chunks of
// rows, then the 16 lanes of a vector, then the chunks), so results do not depend on
// scheduling.  Slabs marked done skip every kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.h"

namespace xbk {

namespace {

constexpr int kGmMaxNv = kGmRestart + 1;

// Fixed-order sum over the 16 lanes of a vector (lanes 16 c .. 16 c + 15).
__device__ __forceinline__ double sum16(double v)
{
    v += __shfl_xor(v, 1, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 8, 16);
    return v;
}
__device__ __forceinline__ double max16(double v)
{
    v = nan_max(v, __shfl_xor(v, 1, 16));
    v = nan_max(v, __shfl_xor(v, 2, 16));
    v = nan_max(v, __shfl_xor(v, 4, 16));
    v = nan_max(v, __shfl_xor(v, 8, 16));
    return v;
}

// part[chunk][i][b] = sum over the chunk's rows of X_i . w for i < nv, X_i = X + i P.
// Grid (nslab, nchunk); thread t: vector col = t / 16 of the slab, lane t % 16 takes
// the entries j = t % 16 + 16 k of each row.
__global__ __launch_bounds__(256) void gm_dots_kernel(GmPanel g, const double* __restrict__ X, int nv,
                                                      const double* __restrict__ w, double* __restrict__ part)
{
    const int slab = blockIdx.x, chunk = blockIdx.y;
    if (g.slab_done[slab]) return;
    const int col = threadIdx.x >> 4, sub = threadIdx.x & 15;
    const int r0 = chunk * g.rows_per_chunk, r1 = min(g.m, r0 + g.rows_per_chunk);
    double acc[kGmMaxNv];
#pragma unroll
    for (int i = 0; i < kGmMaxNv; ++i) acc[i] = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int64_t base = (((int64_t)slab * g.m + r) * 16 + col) * g.n_p;
        for (int j = sub; j < g.n_p; j += 16) {
            const double wv = w[base + j];
#pragma unroll
            for (int i = 0; i < kGmMaxNv; ++i)
                if (i < nv) acc[i] += X[(int64_t)i * g.P + base + j] * wv;
        }
    }
    const int b = 16 * slab + col, Bp = 16 * g.nslab;
#pragma unroll
    for (int i = 0; i < kGmMaxNv; ++i) {
        if (i >= nv) break;
        const double s = sum16(acc[i]);
        if (sub == 0) part[((int64_t)chunk * kGmMaxNv + i) * Bp + b] = s;
    }
}

// out[i][b] = (add ? out[i][b] : 0) + sum over chunks of part[chunk][i][b] (fixed order);
// sqrt_out: out = sqrt of the sum (a norm).  One thread per (i, b).
__global__ __launch_bounds__(256) void gm_finish_dots_kernel(GmPanel g, int nv, const double* __restrict__ part,
                                                             double* __restrict__ out, int ld_out, int add,
                                                             int sqrt_out)
{
    const int Bp = 16 * g.nslab;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nv * Bp) return;
    const int i = e / Bp, b = e % Bp;
    if (g.slab_done[b >> 4]) return;
    double s = 0.0;
    for (int c = 0; c < g.nchunk; ++c) s += part[((int64_t)c * kGmMaxNv + i) * Bp + b];
    if (sqrt_out) s = sqrt(fmax(s, 0.0));
    double* o = out + (int64_t)i * ld_out + b;
    *o = add ? *o + s : s;
}

// w -= sum_{i < nv} coef[i][b] X_i (coef rows of length Bp, coef row stride ld_coef)
__global__ __launch_bounds__(256) void gm_axpy_kernel(GmPanel g, const double* __restrict__ X, int nv,
                                                      const double* __restrict__ coef, int ld_coef,
                                                      double* __restrict__ w)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.P) return;
    const int64_t row = e / g.n_p;                     // (slab m + i) 16 + col
    const int col = (int)(row % 16), slab = (int)(row / (16 * (int64_t)g.m));
    if (g.slab_done[slab]) return;
    const int b = 16 * slab + col;
    double v = w[e];
#pragma unroll
    for (int i = 0; i < kGmMaxNv; ++i) {
        if (i >= nv) break;
        v -= coef[(int64_t)i * ld_coef + b] * X[(int64_t)i * g.P + e];
    }
    w[e] = v;
}

// v = w / s[b] (v = 0 when s[b] is 0 or not finite; v may be w), also rounded to float
// into Rf (the next preconditioner input) when Rf is given
__global__ __launch_bounds__(256) void gm_scale_kernel(GmPanel g, const double* w, const double* __restrict__ s,
                                                       double* v, float* __restrict__ Rf)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= g.P) return;
    const int64_t row = e / g.n_p;
    const int col = (int)(row % 16), slab = (int)(row / (16 * (int64_t)g.m));
    if (g.slab_done[slab]) return;
    const double d = s[16 * slab + col];
    const double x = (d > 0.0 && d < INFINITY) ? w[e] / d : 0.0;
    v[e] = x;
    if (Rf) Rf[e] = (float)x;
}

// Per input vector: minimise |beta e_1 - H y| over y (H: (k+1) x k upper Hessenberg,
// stored H[i][j][b]) by Givens rotations, then back substitution; y[j][b].  A zero
// diagonal after the rotations (breakdown) gives y_j = 0 for that column.
__global__ __launch_bounds__(256) void gm_lsq_kernel(GmPanel g, const double* __restrict__ Hs,
                                                     const double* __restrict__ beta, double* __restrict__ y)
{
    const int Bp = 16 * g.nslab;
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= Bp || g.slab_done[b >> 4]) return;
    constexpr int K = kGmRestart;
    double h[K + 1][K], gv[K + 1], cs[K], sn[K];
    for (int i = 0; i <= K; ++i)
        for (int j = 0; j < K; ++j) h[i][j] = Hs[((int64_t)i * K + j) * Bp + b];
    gv[0] = beta[b];
    for (int i = 1; i <= K; ++i) gv[i] = 0.0;
    for (int j = 0; j < K; ++j) {
        for (int i = 0; i < j; ++i) {
            const double a0 = h[i][j], a1 = h[i + 1][j];
            h[i][j] = cs[i] * a0 + sn[i] * a1;
            h[i + 1][j] = -sn[i] * a0 + cs[i] * a1;
        }
        const double a0 = h[j][j], a1 = h[j + 1][j];
        const double r = hypot(a0, a1);
        cs[j] = r > 0.0 ? a0 / r : 1.0;
        sn[j] = r > 0.0 ? a1 / r : 0.0;
        h[j][j] = r;
        h[j + 1][j] = 0.0;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
    }
    double yy[K];
    for (int j = K - 1; j >= 0; --j) {
        double s = gv[j];
        for (int i = j + 1; i < K; ++i) s -= h[j][i] * yy[i];
        yy[j] = (h[j][j] > 0.0 && std::isfinite(s)) ? s / h[j][j] : 0.0;
    }
    for (int j = 0; j < K; ++j) y[(int64_t)j * Bp + b] = yy[j];
}

// u += sum_j y[j][b] Z_j; part[chunk][0][b] = max |d|, part[chunk][1][b] = max |u| over
// the chunk's rows.  Grid (nslab, nchunk) as the dots.
__global__ __launch_bounds__(256) void gm_update_kernel(GmPanel g, const double* __restrict__ Z,
                                                        const double* __restrict__ y, double* __restrict__ u,
                                                        double* __restrict__ part)
{
    const int slab = blockIdx.x, chunk = blockIdx.y;
    if (g.slab_done[slab]) return;
    const int col = threadIdx.x >> 4, sub = threadIdx.x & 15;
    const int b = 16 * slab + col, Bp = 16 * g.nslab;
    double yy[kGmRestart];
#pragma unroll
    for (int j = 0; j < kGmRestart; ++j) yy[j] = y[(int64_t)j * Bp + b];
    const int r0 = chunk * g.rows_per_chunk, r1 = min(g.m, r0 + g.rows_per_chunk);
    double dmax = 0.0, umax = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int64_t base = (((int64_t)slab * g.m + r) * 16 + col) * g.n_p;
        for (int j = sub; j < g.n_p; j += 16) {
            double d = 0.0;
#pragma unroll
            for (int k = 0; k < kGmRestart; ++k) d += yy[k] * Z[(int64_t)k * g.P + base + j];
            const double x = u[base + j] + d;
            u[base + j] = x;
            dmax = nan_max(dmax, fabs(d));
            umax = nan_max(umax, fabs(x));
        }
    }
    dmax = max16(dmax);
    umax = max16(umax);
    if (sub == 0) {
        part[((int64_t)chunk * kGmMaxNv + 0) * Bp + b] = dmax;
        part[((int64_t)chunk * kGmMaxNv + 1) * Bp + b] = umax;
    }
}

// One thread per slab: the slab is done when every real vector's correction max |d|
// is <= tol max |u| (or not finite: then it stops and reports); outer step `it`.
__global__ __launch_bounds__(256) void gm_converge_kernel(GmPanel g, int B, const double* __restrict__ part,
                                                         double tol, int it, int last, int* __restrict__ flags)
{
    const int slab = blockIdx.x * 256 + threadIdx.x;
    if (slab >= g.nslab || g.slab_done[slab]) return;
    const int Bp = 16 * g.nslab;
    bool all = true, bad = false;
    for (int col = 0; col < 16; ++col) {
        const int b = 16 * slab + col;
        if (b >= B) break;
        double dm = 0.0, um = 0.0;
        for (int c = 0; c < g.nchunk; ++c) {
            dm = nan_max(dm, part[((int64_t)c * kGmMaxNv + 0) * Bp + b]);
            um = nan_max(um, part[((int64_t)c * kGmMaxNv + 1) * Bp + b]);
        }
        if (!std::isfinite(dm) || !std::isfinite(um)) bad = true;
        if (!(dm <= tol * um)) all = false;
    }
    if (all || bad || last) {
        g.slab_done[slab] = 1;
        g.slab_final[slab] = 0;
        atomicMax(flags + kIrIters, it + 1);
        if (!all) atomicOr(flags + kErrConv, 1);
    }
}

// Iout[b][j] = g_sense u[row m - 1][j] of the final solution
__global__ __launch_bounds__(256) void gm_currents_kernel(GmPanel g, int B, int n, double g_sense,
                                                          const double* __restrict__ u, double* __restrict__ Iout)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= B * n) return;
    const int b = e / n, j = e % n, slab = b >> 4, col = b & 15;
    Iout[e] = g_sense * u[(((int64_t)slab * g.m + g.m - 1) * 16 + col) * g.n_p + j];
}

// dst[i][b] += src[i][b] for i < nv (rows of Bp values, strides ld_dst, ld_src)
__global__ __launch_bounds__(256) void gm_add_kernel(GmPanel g, int nv, const double* __restrict__ src, int ld_src,
                                                     double* __restrict__ dst, int ld_dst)
{
    const int Bp = 16 * g.nslab;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nv * Bp) return;
    const int i = e / Bp, b = e % Bp;
    if (g.slab_done[b >> 4]) return;
    dst[(int64_t)i * ld_dst + b] += src[(int64_t)i * ld_src + b];
}

__global__ __launch_bounds__(256) void gm_fill_kernel(double* __restrict__ x, int64_t count, double v)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) x[e] = v;
}

unsigned grid_of(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

}  // namespace xbk

using xbk::GmPanel;

hipError_t xbk_gm_dots(const GmPanel& g, const double* X, int nv, const double* w, double* part, double* out,
                       int ld_out, bool add, bool sqrt_out, hipStream_t s)
{
    if (nv < 1 || nv > xbk::kGmRestart + 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xbk::gm_dots_kernel, dim3(g.nslab, g.nchunk), dim3(256), 0, s, g, X, nv, w, part);
    hipLaunchKernelGGL(xbk::gm_finish_dots_kernel, dim3(xbk::grid_of((int64_t)nv * 16 * g.nslab)), dim3(256), 0, s,
                       g, nv, part, out, ld_out, add ? 1 : 0, sqrt_out ? 1 : 0);
    return hipGetLastError();
}

hipError_t xbk_gm_axpy(const GmPanel& g, const double* X, int nv, const double* coef, int ld_coef, double* w,
                       hipStream_t s)
{
    if (nv < 1 || nv > xbk::kGmRestart + 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xbk::gm_axpy_kernel, dim3(xbk::grid_of(g.P)), dim3(256), 0, s, g, X, nv, coef, ld_coef, w);
    return hipGetLastError();
}

hipError_t xbk_gm_scale(const GmPanel& g, const double* w, const double* sc, double* v, float* Rf, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::gm_scale_kernel, dim3(xbk::grid_of(g.P)), dim3(256), 0, s, g, w, sc, v, Rf);
    return hipGetLastError();
}

hipError_t xbk_gm_lsq(const GmPanel& g, const double* Hs, const double* beta, double* y, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::gm_lsq_kernel, dim3(xbk::grid_of(16 * (int64_t)g.nslab)), dim3(256), 0, s, g, Hs, beta,
                       y);
    return hipGetLastError();
}

hipError_t xbk_gm_update(const GmPanel& g, const double* Z, const double* y, double* u, double* part, int B,
                         double tol, int it, bool last, int* flags, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::gm_update_kernel, dim3(g.nslab, g.nchunk), dim3(256), 0, s, g, Z, y, u, part);
    hipLaunchKernelGGL(xbk::gm_converge_kernel, dim3(xbk::grid_of(g.nslab)), dim3(256), 0, s, g, B, part, tol, it,
                       last ? 1 : 0, flags);
    return hipGetLastError();
}

hipError_t xbk_gm_currents(const GmPanel& g, int B, int n, double g_sense, const double* u, double* Iout,
                           hipStream_t s)
{
    hipLaunchKernelGGL(xbk::gm_currents_kernel, dim3(xbk::grid_of((int64_t)B * n)), dim3(256), 0, s, g, B, n,
                       g_sense, u, Iout);
    return hipGetLastError();
}

hipError_t xbk_gm_fill(double* x, int64_t count, double v, hipStream_t s)
{
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(xbk::gm_fill_kernel, dim3((unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096)),
                       dim3(256), 0, s, x, count, v);
    return hipGetLastError();
}

hipError_t xbk_gm_add(const GmPanel& g, int nv, const double* src, int ld_src, double* dst, int ld_dst, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::gm_add_kernel, dim3(xbk::grid_of((int64_t)nv * 16 * g.nslab)), dim3(256), 0, s, g, nv,
                       src, ld_src, dst, ld_dst);
    return hipGetLastError();
}

// Solution diagnostics and test hooks of a plan.
//
// backward_error_kernel: the normwise backward error of node voltages v for the
// nodal system A v = b of Sec. II.A (stamps of Eqs. 5-7, paper order of Sec. II.B),
//     eta = ||b - A v||_inf / (||A||_inf ||v||_inf + ||b||_inf),
// per input vector, with the residual formed node by node from the stamps:
//     WL(i,j):  t_ij w_ij - g_wl (w_i,j-1 + w_i,j+1) - G_ij u_ij - [j = 0] g_src V_i
//     BL(i,j):  q_ij u_ij - G_ij w_ij - g_bl (u_i-1,j + u_i+1,j)
// (neighbours outside the crossbar are absent), t_ij = G_ij + (j = 0 ? g_src : g_wl)
// + (j < n-1 ? g_wl : 0), q_ij = G_ij + (i > 0 ? g_bl : 0) + (i < m-1 ? g_bl : g_sense),
// and ||A||_inf the largest absolute row sum.  One workgroup per input vector walks
// the crossbar rows; each thread owns columns j = tid + 256 c and keeps the bit-line
// voltages of the two rows above in registers, while the word-line voltages of the
// current row pass through LDS for the neighbours j -/+ 1.  The batch maximum goes to
// the plan's diagnostics word by an integer atomic max on the (non-negative) bits.
//
// shift_diag_kernel: subtracts a shift from every diagonal entry of the condensed
// blocks E_i (a test hook that makes the factor meet non-positive pivots).
//
// For a plan in reciprocal ordering the kernel runs on the crossbar as given (m, n,
// resistances, V and node voltages in its order), reading its conductances from the
// reciprocal crossbar's array.
#include <algorithm>

#include "common.h"

namespace xbk {

constexpr int kBeThreads = 256;
constexpr int kBeCols = 4;            // columns per thread: n <= 1024

__global__ __launch_bounds__(kBeThreads) void backward_error_kernel(BackErrArgs a)
{
    __shared__ double wrow[2][kBeCols * kBeThreads];
    __shared__ double red[3][kBeThreads / 64];
    const int m = a.m, n = a.n, b = blockIdx.x, t = threadIdx.x;
    const double gw = a.g_wl, gb = a.g_bl, gs = a.g_src, gt = a.g_sense;
    const double* v = a.node_v + (int64_t)b * 2 * m * n;
    const double* Vb = a.V + (int64_t)b * m;
    double u1[kBeCols], u2[kBeCols], w1[kBeCols], G1[kBeCols];   // row i-1: u, w, G; u2: row i-2
    double rmax = 0.0, vmax = 0.0, amax = 0.0, bmax = 0.0;
    auto keep = [](double& acc, double x) { acc = (x > acc || x != x) ? x : acc; };
#pragma unroll
    for (int c = 0; c < kBeCols; ++c) u1[c] = u2[c] = w1[c] = G1[c] = 0.0;
    for (int i = 0; i <= m; ++i) {
        double* wr = wrow[i & 1];
        double w0[kBeCols], u0[kBeCols], G0[kBeCols];
        if (i < m) {
#pragma unroll
            for (int c = 0; c < kBeCols; ++c) {
                const int j = t + kBeThreads * c;
                w0[c] = u0[c] = G0[c] = 0.0;
                if (j < n) {
                    typedef double d2v __attribute__((ext_vector_type(2)));
                    const d2v x = *reinterpret_cast<const d2v*>(v + 2 * ((int64_t)i * n + j));
                    w0[c] = x[0];
                    u0[c] = x[1];
                    G0[c] = a.rev ? a.G[(int64_t)(n - 1 - j) * m + (m - 1 - i)] : a.G[(int64_t)i * n + j];
                    wr[j] = x[0];
                    keep(vmax, fabs(x[0]));
                    keep(vmax, fabs(x[1]));
                }
            }
            if (t == 0) keep(bmax, fabs(gs * Vb[i]));
        }
        lds_barrier();
#pragma unroll
        for (int c = 0; c < kBeCols; ++c) {
            const int j = t + kBeThreads * c;
            if (j >= n) continue;
            if (i < m) {
                // word-line node (i, j)
                const double gl = (j == 0) ? gs : gw, gr = (j < n - 1) ? gw : 0.0;
                const double tij = G0[c] + gl + gr;
                double r = (j == 0 ? gs * Vb[i] : 0.0) - tij * w0[c] + G0[c] * u0[c];
                if (j > 0) r += gw * wr[j - 1];
                if (j < n - 1) r += gw * wr[j + 1];
                keep(rmax, fabs(r));
                keep(amax, tij + G0[c] + (j > 0 ? gw : 0.0) + (j < n - 1 ? gw : 0.0));
            }
            if (i > 0) {
                // bit-line node (i-1, j): needs the bit lines of rows i-2, i-1, i
                const int ib = i - 1;
                const double up = (ib > 0) ? gb : 0.0, dn = (ib < m - 1) ? gb : gt;
                const double q = G1[c] + up + dn;
                double r = G1[c] * w1[c] - q * u1[c];
                if (ib > 0) r += gb * u2[c];
                if (ib < m - 1) r += gb * u0[c];
                keep(rmax, fabs(r));
                keep(amax, q + G1[c] + up + (ib < m - 1 ? gb : 0.0));
            }
        }
#pragma unroll
        for (int c = 0; c < kBeCols; ++c) {
            u2[c] = u1[c];
            u1[c] = (i < m) ? u0[c] : 0.0;
            w1[c] = (i < m) ? w0[c] : 0.0;
            G1[c] = (i < m) ? G0[c] : 0.0;
        }
    }
    // workgroup maxima of |r|, |v| and the row sums
    double x[3] = {rmax, vmax, amax};
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(x[k], off);
            x[k] = (o > x[k] || o != o) ? o : x[k];
        }
    if ((t & 63) == 0)
        for (int k = 0; k < 3; ++k) red[k][t >> 6] = x[k];
    __syncthreads();
    if (t == 0) {
        for (int k = 0; k < 3; ++k)
            for (int q = 1; q < kBeThreads / 64; ++q) x[k] = (red[k][q] > x[k] || red[k][q] != red[k][q]) ? red[k][q] : x[k];
        const double den = x[2] * x[1] + bmax;
        const double eta = den > 0.0 ? x[0] / den : (x[0] > 0.0 ? __builtin_inf() : x[0]);
        const double e = (eta != eta) ? __builtin_nan("") : fabs(eta);
        atomicMax(a.diag + kDiagBackErr, __builtin_bit_cast(unsigned long long, e));
    }
}

template <typename T>
__global__ void shift_diag_kernel(void* E, int m, int n, int n_p, double shift)
{
    T* e = reinterpret_cast<T*>(E);
    const int64_t total = (int64_t)m * n;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x / n;
        const int k = (int)(x - i * n);
        e[i * n_p * n_p + frg<T>(k, k, n_p)] -= (T)shift;
    }
}

__global__ void reset_diag_kernel(unsigned long long* diag, int which)
{
    if (threadIdx.x == 0) {
        if (which & 1) diag[kDiagMinPivot] = kPivotKeyInf;
        if (which & 2) diag[kDiagBackErr] = 0ull;
    }
}

}  // namespace xbk

hipError_t xbk_launch_backward_error(const xbk::BackErrArgs& a, hipStream_t s)
{
    if (a.n > xbk::kBeCols * xbk::kBeThreads || a.B < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xbk::backward_error_kernel, dim3(a.B), dim3(xbk::kBeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t xbk_launch_shift_diag(void* E, bool fp32, int m, int n, int n_p, double shift, hipStream_t s)
{
    const int64_t total = (int64_t)m * n;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    if (fp32)
        hipLaunchKernelGGL(xbk::shift_diag_kernel<float>, dim3(grid), dim3(256), 0, s, E, m, n, n_p, shift);
    else
        hipLaunchKernelGGL(xbk::shift_diag_kernel<double>, dim3(grid), dim3(256), 0, s, E, m, n, n_p, shift);
    return hipGetLastError();
}

hipError_t xbk_launch_reset_diag(unsigned long long* diag, int which, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::reset_diag_kernel, dim3(1), dim3(64), 0, s, diag, which);
    return hipGetLastError();
}

int xbk_backward_error_max_n() { return xbk::kBeCols * xbk::kBeThreads; }

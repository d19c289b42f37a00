// Batched small crossbars: the output currents of many crossbars of one shape
// (n <= 64 columns), one workgroup per crossbar, the whole solve in one launch.
//
// Per crossbar the method is the one of the large path (Sec. II.A-II.C):
// eliminate each row's word-line nodes (E_i = Q_i - Gam_i T_i^-1 Gam_i, source
// coupling c_i = g_src Gam_i T_i^-1 e_0), then a block LU over the rows.  Here
// the rows are taken top-down in one chain, S_i = E_i - g_bl^2 H_{i-1},
// H_i = S_i^-1, with the forward substitution z_i = H_i (V_i c_i + g_bl z_{i-1})
// run alongside.  The bottom row's forward result is already its solution (the
// back substitution leaves the last row unchanged), so the output currents
// g_sense z_{m-1} need no back substitution and no row block is stored.
//
// Workgroup layout (256 threads, NP x NP blocks padded with identity to NP in
// {16, 32, 64}):
//  * thread k < n walks column k of T_i^-1 with the Thomas recurrences of the
//    word-line chain and writes column k of S_i into LDS;
//  * S_i is inverted in place by Gauss-Jordan elimination without pivoting (S_i
//    is symmetric positive definite); thread t owns the elements e = t + 256 s
//    (two barriers per pivot step: read, then write);
//  * thread b < B keeps z for input vector b in registers and forms the next z
//    from H_i in LDS (every lane reads the same H element: LDS broadcast).
// Two LDS blocks alternate: S_i is built in one while H_{i-1} sits in the other.
// A tile with a conductance that is not finite and positive, or a pivot that is
// not positive, gets NaN currents.
// float64 throughout.  The float64 vector units of this part run at the
// float64 matrix-core rate, so the n x n x B product per row stays on them.
#include <climits>
#include <cmath>
#include <cstdint>

#include "tiles.h"

namespace {

constexpr int kTileThreads = 256;

struct TileArgs {
    int m, n, B;
    double g_wl, g_bl, g_src, g_sense;
    const double* G;    // [T][m][n]
    const double* V;    // [T][B][m]
    double* I;          // [T][B][n]
};

template <int NP>
__global__ __launch_bounds__(kTileThreads) void tile_currents_kernel(TileArgs a)
{
    constexpr int LD = NP;     // row stride: every cross-lane LDS access is a row or a broadcast
    constexpr int PER = NP * NP / kTileThreads > 0 ? NP * NP / kTileThreads : 1;
    __shared__ double blk[2][NP * LD];
    __shared__ double gr[NP], cr[NP], piv[NP];
    __shared__ int bad;

    const int tid = threadIdx.x;
    const int m = a.m, n = a.n, B = a.B;
    const int64_t t = blockIdx.x;
    const double* G = a.G + t * m * n;
    const double* V = a.V + t * B * m;
    double* I = a.I + t * B * n;
    const double gw = a.g_wl, gb = a.g_bl;
    if (tid == 0) bad = 0;
    __syncthreads();

    double z[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) z[k] = 0.0;

    for (int i = 0; i < m; ++i) {
        double* S = blk[i & 1];
        const double* Hp = blk[(i & 1) ^ 1];
        // ---- row data and the pivots of the word-line chain (excess form, no subtraction):
        // e_0 = G_0 + g_src, e_j = G_j + g_wl e_{j-1} / p_{j-1}, p_j = e_j + g_wl [j < n-1]
        if (tid < n) {
            const double g = G[(int64_t)i * n + tid];
            gr[tid] = g;
            if (!(g > 0.0 && g <= 1e300)) bad = 1;
        }
        __syncthreads();
        if (tid == 0) {
            double e = gr[0] + a.g_src;
            piv[0] = e + (n > 1 ? gw : 0.0);
            for (int j = 1; j < n; ++j) {
                e = gr[j] + gw * e / piv[j - 1];
                piv[j] = e + (j < n - 1 ? gw : 0.0);
            }
        }
        __syncthreads();
        // ---- column k of T_i^-1 (thread k): forward y_j = [j = k] + (g_wl / p_{j-1}) y_{j-1},
        // back x_j = (y_j + g_wl x_{j+1}) / p_j, kept in column k of S
        if (tid < n) {
            const int k = tid;
            double y = 0.0;
            for (int j = k; j < n; ++j) {
                y = (j == k ? 1.0 : 0.0) + (j > k ? gw / piv[j - 1] * y : 0.0);
                S[j * LD + k] = y;
            }
            for (int j = 0; j < k; ++j) S[j * LD + k] = 0.0;
            double x = 0.0;
            for (int j = n - 1; j >= 0; --j) {
                x = (S[j * LD + k] + (j < n - 1 ? gw * x : 0.0)) / piv[j];
                S[j * LD + k] = x;
            }
        }
        __syncthreads();
        // ---- S_i = diag(q_i) - Gam T^-1 Gam - g_bl^2 H_{i-1}, identity on the padding;
        // c_i = g_src Gam T^-1 e_0
        {
            const double below = (i < m - 1) ? gb : a.g_sense;
            const double above = (i > 0) ? gb : 0.0;
            const double g2 = gb * gb;
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const int e = tid + kTileThreads * s;
                if (e < NP * NP) {
                    const int r = e / NP, c = e % NP;
                    double v;
                    if (r < n && c < n) {
                        v = -gr[r] * S[r * LD + c] * gr[c];
                        if (r == c) v += gr[r] + above + below;
                        if (i > 0) v -= g2 * Hp[r * LD + c];
                    } else {
                        v = (r == c) ? 1.0 : 0.0;
                    }
                    if (c == 0 && r < n) cr[r] = a.g_src * gr[r] * S[r * LD];
                    // all reads of column c above were this thread's own column-0 or (r, c) entry
                    // except S[r][0] for c == 0, which is the same element: safe in place
                    S[r * LD + c] = v;
                }
            }
        }
        __syncthreads();
        // ---- H_i = S_i^-1 in place (Gauss-Jordan, no pivoting)
        for (int k = 0; k < n; ++k) {
            const double p = S[k * LD + k];
            double f[PER], rk[PER];
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const int e = tid + kTileThreads * s;
                const int r = e / NP, c = e % NP;
                f[s] = (e < NP * NP) ? S[r * LD + k] : 0.0;
                rk[s] = (e < NP * NP) ? S[k * LD + c] : 0.0;
            }
            if (tid == 0 && !(p > 0.0 && p <= 1e300)) bad = 1;
            __syncthreads();
            const double pinv = 1.0 / p;
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const int e = tid + kTileThreads * s;
                if (e < NP * NP) {
                    const int r = e / NP, c = e % NP;
                    const double nk = (c == k ? 1.0 : rk[s]) * pinv;     // new row k, column c
                    S[r * LD + c] = (r == k) ? nk : ((c == k ? 0.0 : S[r * LD + c]) - f[s] * nk);
                }
            }
            __syncthreads();
        }
        // ---- z <- H_i (V_i c_i + g_bl z) for this thread's input vector
        if (tid < B) {
            const double vi = V[(int64_t)tid * m + i];
            double y[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) y[k] = (k < n ? vi * cr[k] : 0.0) + gb * z[k];
#pragma unroll
            for (int r = 0; r < NP; ++r) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < NP; k += 2) {
                    const double2 h = *reinterpret_cast<const double2*>(&S[r * LD + k]);
                    acc += h.x * y[k] + h.y * y[k + 1];
                }
                z[r] = acc;
            }
        }
        __syncthreads();          // H_i stays in this block for the next row's S_{i+1}
    }
    if (tid < B) {
        const bool fail = bad != 0;
#pragma unroll
        for (int j = 0; j < NP; ++j)           // unrolled: z stays in registers
            if (j < n) I[(int64_t)tid * n + j] = fail ? NAN : a.g_sense * z[j];
    }
}

}  // namespace

hipError_t xbk_launch_tile_currents(int T, int m, int n, int B, double g_wl, double g_bl, double g_src,
                                    double g_sense, const double* G, const double* V, double* I, hipStream_t s)
{
    if (T < 1 || m < 1 || n < 1 || n > 64 || B < 1 || B > kTileThreads || !G || !V || !I)
        return hipErrorInvalidValue;
    TileArgs a{m, n, B, g_wl, g_bl, g_src, g_sense, G, V, I};
    const dim3 grid((unsigned)T), block(kTileThreads);
    if (n <= 16)
        hipLaunchKernelGGL(tile_currents_kernel<16>, grid, block, 0, s, a);
    else if (n <= 32)
        hipLaunchKernelGGL(tile_currents_kernel<32>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(tile_currents_kernel<64>, grid, block, 0, s, a);
    return hipGetLastError();
}

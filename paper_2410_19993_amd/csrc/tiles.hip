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
// Workgroup layout (256 threads = 4 waves, blocks padded with identity to NP in
// {16, 32, 64}, BS = NP / 16):
//  * thread k < n walks column k of T_i^-1 with the Thomas recurrences of the
//    word-line chain (reciprocal pivots, so only multiplications) into LDS;
//  * thread t = 16 br + bc holds the BS x BS block (br, bc) of S_i in registers
//    and inverts S_i in place with the others by Gauss-Jordan elimination
//    without pivoting (S_i is SPD), four pivots per step: only the four pivot
//    rows and columns go through LDS (double-buffered, one barrier per step);
//  * the product H_i Y runs on the float64 matrix cores: wave w owns input
//    vectors 64 w .. 64 w + 63 as four groups of 16, and keeps their forward
//    results in the accumulator layout (item v of lane l = 16 q + c is row
//    q + 4v of a 16-row tile, vector c of a group).  That is also the B-operand
//    layout of the next row's product, so the forward results never move.  The
//    A operand, H_i, is read from LDS along rows (H_i is symmetric).
// Two LDS blocks alternate: T_i^-1, then H_i, in one, while H_{i-1} sits in the
// other.  A tile with a conductance that is not finite and positive, or a pivot
// that is not positive, gets NaN currents.  float64 throughout.
#include <climits>
#include <cmath>
#include <cstdint>

#include "tiles.h"

namespace {

constexpr int kTileThreads = 256;

typedef double dv4 __attribute__((ext_vector_type(4)));

// 1 / x for the positive normal pivots here: the hardware reciprocal estimate
// refined by two Newton-Raphson steps r <- r + r (1 - x r), each of which squares
// the relative error (full double precision after the second)
__device__ inline double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// A crossbar's B input vectors may be split over gridDim.y workgroups (Bp each, the
// last one fewer): each redoes the crossbar's factorization and forward-substitutes its
// own vectors, trading repeated elimination for more workgroups in flight.
struct TileArgs {
    int m, n, B, Bp;
    int unit;           // 1: input vector b is the unit vector e_b (V is not read)
    double g_wl, g_bl, g_src, g_sense;
    const double* G;    // [T][m][n]
    const double* V;    // [T][B][m]
    double* I;          // [T][B][n]
};

template <int NP>
__global__ __launch_bounds__(kTileThreads) void tile_currents_kernel(TileArgs a)
{
    constexpr int LD = NP;                             // row stride of the LDS blocks
    constexpr int BS = NP / 16;                        // register block edge of the elimination
    constexpr int NT = NP / 16;                        // 16-row tiles of the product
    __shared__ __align__(16) double blk[2][NP * LD];
    __shared__ __align__(16) double rowb[2][4][NP], colb[2][4][NP];   // [buffer][pivot][index]
    __shared__ double gr[NP], cr[NP], piv[NP], rpiv[NP];
    __shared__ int bad;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int q = lane >> 4, l16 = lane & 15;
    const int br = tid >> 4, bc = tid & 15;
    const int m = a.m, n = a.n;
    const int64_t t = blockIdx.x;
    const int b0 = (int)blockIdx.y * a.Bp;                 // first vector of this workgroup
    const int B = min(a.Bp, a.B - b0);                      // vectors of this workgroup
    const double* G = a.G + t * m * n;
    const double* V = a.V + (t * a.B + b0) * m;
    double* I = a.I + (t * a.B + b0) * n;
    const double gw = a.g_wl, gb = a.g_bl;
    if (tid == 0) bad = 0;
    __syncthreads();

    // forward results of vectors 64 w + 16 g + l16: z[tile][g] item v = row 16 tile + q + 4 v
    dv4 z[NT][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int g = 0; g < 4; ++g) z[tt][g] = dv4{0.0, 0.0, 0.0, 0.0};

    for (int i = 0; i < m; ++i) {
        double* Tb = blk[i & 1];                       // T_i^-1, then H_i
        const double* Hp = blk[(i & 1) ^ 1];           // H_{i-1}
        // ---- row data; pivots of the word-line chain (excess form, no subtraction):
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
            rpiv[0] = recip(piv[0]);
            for (int j = 1; j < n; ++j) {
                e = gr[j] + gw * e * rpiv[j - 1];
                piv[j] = e + (j < n - 1 ? gw : 0.0);
                rpiv[j] = recip(piv[j]);
            }
        }
        __syncthreads();
        // ---- column k of T_i^-1 (thread k): y_j = [j = k] + g_wl y_{j-1} / p_{j-1},
        // x_j = (y_j + g_wl x_{j+1}) / p_j
        if (tid < n) {
            const int k = tid;
            double y = 0.0;
            for (int j = k; j < n; ++j) {
                y = (j == k) ? 1.0 : gw * rpiv[j - 1] * y;
                Tb[j * LD + k] = y;
            }
            for (int j = 0; j < k; ++j) Tb[j * LD + k] = 0.0;
            double x = 0.0;
            for (int j = n - 1; j >= 0; --j) {
                x = (Tb[j * LD + k] + (j < n - 1 ? gw * x : 0.0)) * rpiv[j];
                Tb[j * LD + k] = x;
            }
        }
        __syncthreads();
        // ---- S_i = diag(q_i) - Gam T^-1 Gam - g_bl^2 H_{i-1} (identity on the padding) into
        // this thread's register block; c_i = g_src Gam T^-1 e_0 (zero on the padding)
        double s[BS][BS];
        {
            const double below = (i < m - 1) ? gb : a.g_sense;
            const double above = (i > 0) ? gb : 0.0;
            const double g2 = gb * gb;
#pragma unroll
            for (int ii = 0; ii < BS; ++ii) {
                const int r = BS * br + ii;
#pragma unroll
                for (int jj = 0; jj < BS; ++jj) {
                    const int c = BS * bc + jj;
                    double v = (r == c) ? 1.0 : 0.0;
                    if (r < n && c < n) {
                        v = -gr[r] * Tb[r * LD + c] * gr[c];
                        if (r == c) v += gr[r] + above + below;
                        if (i > 0) v -= g2 * Hp[r * LD + c];
                    }
                    s[ii][jj] = v;
                }
                if (bc == 0) cr[r] = (r < n) ? a.g_src * gr[r] * Tb[r * LD] : 0.0;
            }
        }
        // ---- H_i = S_i^-1 (Gauss-Jordan, no pivoting) on the register blocks, four pivots
        // K = {k .. k+3} per step: the 4 x 4 pivot block P = S[K][K] is inverted in
        // registers by every thread, and
        //   S[K][c] <- P^-1 S'[K][c],  S[r][c] <- S'[r][c] - S[r][K] P^-1 S'[K][c]  (r not in K)
        // where S' is S with S[.][K] replaced by the identity columns.  The padding is
        // the identity, so blocks that reach past n stay exact.
        for (int k = 0, step = 0; k < n; k += 4, ++step) {
            const int kb = step & 1;
#pragma unroll
            for (int ii = 0; ii < BS; ++ii) {
                const int r = BS * br + ii;
                if (r >= k && r < k + 4) {
#pragma unroll
                    for (int jj = 0; jj < BS; ++jj) rowb[kb][r - k][BS * bc + jj] = s[ii][jj];
                }
            }
#pragma unroll
            for (int jj = 0; jj < BS; ++jj) {
                const int c = BS * bc + jj;
                if (c >= k && c < k + 4) {
#pragma unroll
                    for (int ii = 0; ii < BS; ++ii) colb[kb][c - k][BS * br + ii] = s[ii][jj];
                }
            }
            __syncthreads();
            double P[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) P[u][v] = rowb[kb][u][k + v];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double pv = P[t][t];
                if (tid == 0 && !(pv > 0.0 && pv <= 1e300)) bad = 1;
                const double rp = recip(pv);
                double row[4], col[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    row[v] = (v == t ? 1.0 : P[t][v]) * rp;
                    col[v] = P[v][t];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) P[u][v] = (u == t) ? row[v] : ((v == t ? 0.0 : P[u][v]) - col[u] * row[v]);
            }
            double f[4][BS], nn[4][BS], keep[BS];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int ii = 0; ii < BS; ++ii) f[t][ii] = colb[kb][t][BS * br + ii];
#pragma unroll
            for (int jj = 0; jj < BS; ++jj) {
                const int c = BS * bc + jj, ck = c - k;
                const bool inK = ck >= 0 && ck < 4;
                double u[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) u[t] = inK ? (ck == t ? 1.0 : 0.0) : rowb[kb][t][c];
#pragma unroll
                for (int t = 0; t < 4; ++t) nn[t][jj] = P[t][0] * u[0] + P[t][1] * u[1] + P[t][2] * u[2] + P[t][3] * u[3];
                keep[jj] = inK ? 0.0 : 1.0;
            }
#pragma unroll
            for (int ii = 0; ii < BS; ++ii) {
                const int rk = BS * br + ii - k;
                const bool inK = rk >= 0 && rk < 4;
#pragma unroll
                for (int jj = 0; jj < BS; ++jj) {
                    double own = nn[0][jj];
#pragma unroll
                    for (int t = 1; t < 4; ++t) own = (rk == t) ? nn[t][jj] : own;
                    const double upd = s[ii][jj] * keep[jj] - f[0][ii] * nn[0][jj] - f[1][ii] * nn[1][jj] -
                                       f[2][ii] * nn[2][jj] - f[3][ii] * nn[3][jj];
                    s[ii][jj] = inK ? own : upd;
                }
            }
        }
        // ---- H_i into LDS (T_i^-1 there is no longer needed)
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < BS; ++ii)
#pragma unroll
            for (int jj = 0; jj < BS; ++jj) Tb[(BS * br + ii) * LD + BS * bc + jj] = s[ii][jj];
        __syncthreads();
        // ---- z <- H_i (V_i c_i + g_bl z) on the matrix cores
        {
            double vi[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int b = 64 * w + 16 * g + l16;
                vi[g] = (b < B) ? (a.unit ? (b0 + b == i ? 1.0 : 0.0) : V[(int64_t)b * m + i]) : 0.0;
            }
            dv4 y[NT][4];
#pragma unroll
            for (int kc = 0; kc < NT; ++kc)
#pragma unroll
                for (int tq = 0; tq < 4; ++tq) {
                    const double ck = cr[16 * kc + q + 4 * tq];
#pragma unroll
                    for (int g = 0; g < 4; ++g) y[kc][g][tq] = vi[g] * ck + gb * z[kc][g][tq];
                }
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
#pragma unroll
                for (int g = 0; g < 4; ++g) z[tt][g] = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kc = 0; kc < NT; ++kc)
#pragma unroll
                    for (int tq = 0; tq < 4; ++tq) {
                        // A operand H[16 tt + l16][16 kc + q + 4 tq], read as its mirror H[k][a]
                        const double h = Tb[(16 * kc + q + 4 * tq) * LD + 16 * tt + l16];
#pragma unroll
                        for (int g = 0; g < 4; ++g)
                            z[tt][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(h, y[kc][g][tq], z[tt][g], 0, 0, 0);
                    }
            }
        }
        __syncthreads();
    }
    const bool fail = bad != 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int b = 64 * w + 16 * g + l16;
        if (b >= B) continue;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * tt + q + 4 * v;
                if (j < n) I[(int64_t)b * n + j] = fail ? NAN : a.g_sense * z[tt][g][v];
            }
    }
}

}  // namespace

hipError_t xbk_launch_tile_currents(int T, int m, int n, int B, double g_wl, double g_bl, double g_src,
                                    double g_sense, const double* G, const double* V, double* I, hipStream_t s,
                                    int block, int split, bool unit)
{
    if (T < 1 || m < 1 || n < 1 || n > 64 || B < 1 || B > kTileThreads || !G || (!V && !unit) || !I)
        return hipErrorInvalidValue;
    if (block == 0) block = n <= 16 ? 16 : n <= 32 ? 32 : 64;
    if ((block != 16 && block != 32 && block != 64) || block < n || split < 1 || split > 4) return hipErrorInvalidValue;
    const int Bp = (B + split - 1) / split;
    const int parts = (B + Bp - 1) / Bp;
    TileArgs a{m, n, B, Bp, unit ? 1 : 0, g_wl, g_bl, g_src, g_sense, G, V, I};
    const dim3 grid((unsigned)T, (unsigned)parts), blk(kTileThreads);
    if (block == 16)
        hipLaunchKernelGGL(tile_currents_kernel<16>, grid, blk, 0, s, a);
    else if (block == 32)
        hipLaunchKernelGGL(tile_currents_kernel<32>, grid, blk, 0, s, a);
    else
        hipLaunchKernelGGL(tile_currents_kernel<64>, grid, blk, 0, s, a);
    return hipGetLastError();
}

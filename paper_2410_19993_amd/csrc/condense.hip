// Assembly and row condensation (nodal equations of Sec. II.A, Eqs. 1-7).
//
// With the unknowns of crossbar row i grouped as [w_i; u_i] (word-line and
// bit-line node voltages of the row), the nodal equations read
//     T_i w_i - Gam_i u_i                   = g_src V_i e_0
//    -Gam_i w_i + Q_i u_i - g_bl (u_{i-1} + u_{i+1}) = 0
// where T_i = tridiag(-g_wl, t_i, -g_wl) couples the word-line nodes,
// Gam_i = diag(G[i][:]) are the devices and Q_i = diag(q_i) the bit-line
// self conductances.  The self conductances are the stamps of Eqs. 5-7:
//     t_ij = G_ij + (j == 0 ? g_src : g_wl) + (j < n-1 ? g_wl : 0)
//     q_ij = G_ij + (i > 0 ? g_bl : 0) + (i < m-1 ? g_bl : g_sense)
// Eliminating w_i (the first half of an LU of the row's 2n x 2n diagonal
// block, word-line nodes first) leaves the n x n bit-line block
//     E_i = Q_i - Gam_i T_i^{-1} Gam_i,   c_i = g_src Gam_i T_i^{-1} e_0,
// and the block-tridiagonal system E_i u_i - g_bl (u_{i-1} + u_{i+1}) = V_i c_i.
//
// T_i^{-1} is formed column by column from the forward and backward pivots
// of T_i, computed without subtractions (T_i is a diagonally dominant
// M-matrix): with excess d_j = p_j - (right conductance),
//     d_0 = G_0 + g_src,  d_j = G_j + g_wl * d_{j-1} / p_{j-1},
// and symmetrically from the right end.  One workgroup per crossbar row.
#include "common.h"

namespace xbk {

// Row k of FRG tile (k >> 4, c) of an n_p x n_p block: the tile's 16 values v[e]
// (e = column within the tile), as 16-byte stores (two values per lane for
// float64: columns q and q+4, q+8 and q+12 of lane 16q + r; four for float32).
template <typename T>
__device__ __forceinline__ void store_tile_row(T* E, int n_p, int k, int c, const double (&v)[16])
{
    T* tile = E + ((int64_t)(k >> 4) * (n_p >> 4) + c) * 256;
    const int r = k & 15;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int l = 16 * q + r;
        if constexpr (sizeof(T) == 8) {
            typedef double d2v __attribute__((ext_vector_type(2)));
            *reinterpret_cast<d2v*>(tile + frg_slot<T>(l, 0)) = d2v{v[q], v[q + 4]};
            *reinterpret_cast<d2v*>(tile + frg_slot<T>(l, 2)) = d2v{v[q + 8], v[q + 12]};
        } else {
            *reinterpret_cast<f4_t*>(tile + frg_slot<T>(l, 0)) =
                f4_t{(float)v[4 * q], (float)v[4 * q + 1], (float)v[4 * q + 2], (float)v[4 * q + 3]};
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void condense_kernel(CondenseArgs a)
{
    extern __shared__ double lds[];
    const int n = a.n, n_p = a.n_p, i = blockIdx.x;
    if (blockIdx.y > 0) {
        // crossbar blockIdx.y of a batch of one shape
        const int64_t t = blockIdx.y, mn = (int64_t)a.m * n;
        a.G += t * mn;
        a.E = reinterpret_cast<T*>(a.E) + t * (int64_t)a.m * n_p * n_p;
        a.c += t * (int64_t)a.m * n_p;
        a.fr += t * mn;
        a.ip += t * mn;
        a.q += t * mn;
        a.Gc += t * mn;
    }
    double* Gs = lds;            // G_ij
    double* fp = Gs + n;         // forward pivots p_j of T_i
    double* fx = fp + n;         // forward excess d_j = p_j - (right link)
    double* bp = fx + n;         // backward pivots pb_j
    double* bx = bp + n;         // backward excess e_j = pb_j - (left link)
    double* dg = bx + n;         // (T^{-1})_jj
    double* rf = dg + n;         // g_wl / p_j   (ratio going up a column of T^{-1})
    double* rb = rf + n;         // g_wl / pb_j  (ratio going down a column)

    const double gw = a.g_wl;
    const double* Grow = a.G + (int64_t)i * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double g = Grow[j];
        if (!(g > 0.0) || !isfinite(g)) {
            atomicOr(a.flags + kErrInput, 1);
            if (a.tile_bad) atomicOr(a.tile_bad + blockIdx.y, 1);
        }
        Gs[j] = g;
        a.Gc[(int64_t)i * n + j] = g;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = Gs[0] + a.g_src;                       // node 0: device + source link
        for (int j = 0; j < n; ++j) {
            if (j > 0) d = Gs[j] + gw * (fx[j - 1] / fp[j - 1]);
            const double p = d + (j < n - 1 ? gw : 0.0);
            fx[j] = d;
            fp[j] = p;
            rf[j] = gw / p;
        }
    } else if (threadIdx.x == 64) {
        double e = Gs[n - 1];                             // last node: device only
        for (int j = n - 1; j >= 0; --j) {
            if (j < n - 1) e = Gs[j] + gw * (bx[j + 1] / bp[j + 1]);
            const double p = e + (j > 0 ? gw : a.g_src);
            bx[j] = e;
            bp[j] = p;
            rb[j] = gw / p;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        // 1/(T^{-1})_kk = G_k + (left link after eliminating 0..k-1) + (right link after k+1..n-1)
        const double left = (k == 0) ? a.g_src : gw * (fx[k - 1] / fp[k - 1]);
        const double right = (k == n - 1) ? 0.0 : gw * (bx[k + 1] / bp[k + 1]);
        dg[k] = 1.0 / (Gs[k] + left + right);
    }
    __syncthreads();

    const double qb_up = (i > 0) ? a.g_bl : 0.0;
    const double qb_dn = (i < a.m - 1) ? a.g_bl : a.g_sense;
    T* E = reinterpret_cast<T*>(a.E) + (int64_t)i * n_p * n_p;
    const int ct = n_p >> 4;
    // E is symmetric, so thread k produces row k of E as it walks column k of
    // T^{-1}; a tile's 16 values of the row are kept in registers and written
    // with 16-byte stores, so the 16 threads of a tile row fill whole lines.
    for (int k = threadIdx.x; k < n_p; k += blockDim.x) {
        double v[16];
        if (k >= n) {
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = 0.0;
            for (int c = 0; c < ct; ++c) store_tile_row<T>(E, n_p, k, c, v);
            a.c[(int64_t)i * n_p + k] = 0.0;
            continue;
        }
        const int ck = k >> 4, kk = k & 15;
        const double Gk = Gs[k];
        const double qk = Gk + qb_up + qb_dn;
        double home[16];
        // up column k within the home tile: x_j = x_{j+1} g_wl / p_j, j = k-1 .. 16 ck
        double x = dg[k];
#pragma unroll
        for (int e = 15; e >= 0; --e) {
            const int j = 16 * ck + e;
            if (e < kk) {
                x *= rf[j];
                home[e] = -(Gs[j] * x * Gk);
            } else {
                home[e] = 0.0;
            }
        }
        home[kk] = qk - Gk * dg[k] * Gk;
        // the tiles to the left, right to left
        for (int c = ck - 1; c >= 0; --c) {
#pragma unroll
            for (int e = 15; e >= 0; --e) {
                const int j = 16 * c + e;
                x *= rf[j];
                v[e] = -(Gs[j] * x * Gk);
            }
            store_tile_row<T>(E, n_p, k, c, v);
        }
        a.c[(int64_t)i * n_p + k] = a.g_src * Gk * x;   // x = (T^{-1})_{0k} = (T^{-1})_{k0}
        // down column k: x_j = x_{j-1} g_wl / pb_j, j = k+1 .. n-1 (zero on the padding)
        x = dg[k];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int j = 16 * ck + e;
            if (e > kk && j < n) {
                x *= rb[j];
                home[e] = -(Gs[j] * x * Gk);
            }
        }
        store_tile_row<T>(E, n_p, k, ck, home);
        for (int c = ck + 1; c < ct; ++c) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int j = 16 * c + e;
                if (j < n) {
                    x *= rb[j];
                    v[e] = -(Gs[j] * x * Gk);
                } else {
                    v[e] = 0.0;
                }
            }
            store_tile_row<T>(E, n_p, k, c, v);
        }
        a.q[(int64_t)i * n + k] = qk;
        a.fr[(int64_t)i * n + k] = (k == 0) ? 0.0 : rf[k - 1];
        a.ip[(int64_t)i * n + k] = 1.0 / fp[k];
    }
}

}  // namespace xbk

hipError_t xbk_launch_condense(const xbk::CondenseArgs& a, bool fp32, hipStream_t s, int batch)
{
    const size_t lds = 8 * (size_t)a.n * sizeof(double);
    if (fp32)
        hipLaunchKernelGGL(xbk::condense_kernel<float>, dim3(a.m, batch), dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(xbk::condense_kernel<double>, dim3(a.m, batch), dim3(256), lds, s, a);
    return hipGetLastError();
}

// Float64 matrix-core product for the transfer-matrix shortcut.  The crossbar
// is a linear network: the nodal system of Sec. II.A has a right-hand side that
// is linear in the word-line sources, so the output currents of any batch are
// the input voltages times the m x n matrix of output currents per unit input.
//
// Tiling (gfx950, wave64): a workgroup of 4 waves owns a 128 x 64 block of I
// and walks the contraction index k in chunks of 16.  Each chunk of V
// (128 x 16) and of T (16 x 64) is staged in LDS in matrix-core operand order:
// 16 x 16 tiles, lane l = 16q + r holding the four values k = 4q + t,
// t = 0..3, so every lane fetches its operands for four v_mfma_f64_16x16x4f64
// steps with two 16-byte LDS loads.  Wave w computes rows 32w..32w+31 against
// all 64 columns (2 x 4 output tiles, 32 float64 accumulators per lane).  The
// next chunk is loaded from global memory into registers while the matrix
// cores run and written to the other LDS buffer: one barrier per chunk.
//
// XCD-aware launch: workgroups are dealt to the 8 XCDs round-robin.  When the
// row panels divide by 8, each XCD gets a contiguous range of row panels with
// all their column tiles, so one XCD reads each panel of V from HBM and T,
// which every workgroup reads, stays in each XCD's L2.
#include <climits>
#include <cstdint>

#include "transfer.h"

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 128;     // rows of I per workgroup
constexpr int kBN = 64;      // columns of I per workgroup
constexpr int kBK = 16;      // contraction chunk
constexpr int kThreads = 256;

// p[0..valid-1] into x, zeros beyond; one pair of 16-byte loads when allowed
template <bool VEC>
__device__ inline void load4(const double* p, int valid, double (&x)[4])
{
    if (VEC && valid == 4) {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        x[0] = a.x;
        x[1] = a.y;
        x[2] = b.x;
        x[3] = b.y;
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = t < valid ? p[t] : 0.0;
    }
}

__device__ inline int clamp4(int v) { return v < 0 ? 0 : (v > 4 ? 4 : v); }

// VEC: m and n even and V, T 16-byte aligned, so every 4-wide piece starts 16-byte aligned
template <bool VEC>
__global__ __launch_bounds__(kThreads) void transfer_apply_kernel(
    const double* __restrict__ V, const double* __restrict__ T, double* __restrict__ I,
    int B, int m, int n, int col_tiles, int xcd_rows)
{
    __shared__ __align__(16) double la[2][8 * 256];   // V chunk: [row tile][lane][t]
    __shared__ __align__(16) double lb[2][4 * 256];   // T chunk: [column tile][lane][t]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int bid = blockIdx.x;
    int rp, ct;
    if (xcd_rows > 0) {
        const int xcd = bid & 7, local = bid >> 3;
        rp = xcd * xcd_rows + local / col_tiles;
        ct = local % col_tiles;
    } else {
        rp = bid / col_tiles;
        ct = bid % col_tiles;
    }
    const int64_t r0 = (int64_t)rp * kBM;
    const int c0 = ct * kBN;

    // this thread's share of a chunk: two 4-wide pieces of V rows, one 4-wide piece of a T row
    int a_row[2], a_q[2];
    bool a_ok[2];
    const double* a_src[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int g = tid + kThreads * e;
        a_row[e] = g >> 2;
        a_q[e] = g & 3;
        a_ok[e] = r0 + a_row[e] < B;
        a_src[e] = V + (a_ok[e] ? (r0 + a_row[e]) * (int64_t)m : 0) + 4 * a_q[e];
    }
    const int b_kk = tid >> 4, b_c = (tid & 15) * 4;
    const int b_cols = clamp4(n - (c0 + b_c));
    const double* b_src = T + c0 + b_c;

    double ra[2][4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 2; ++e)
            load4<VEC>(a_src[e] + k0, a_ok[e] ? clamp4(m - (k0 + 4 * a_q[e])) : 0, ra[e]);
        const int k = k0 + b_kk;
        load4<VEC>(b_src + (k < m ? (int64_t)k * n : 0), k < m ? b_cols : 0, rb);
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int rt = a_row[e] >> 4, rr = a_row[e] & 15;
            double* d = &la[buf][rt * 256 + (16 * a_q[e] + rr) * 4];
            *reinterpret_cast<double2*>(d) = double2{ra[e][0], ra[e][1]};
            *reinterpret_cast<double2*>(d + 2) = double2{ra[e][2], ra[e][3]};
        }
        const int q = b_kk >> 2, t = b_kk & 3;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = b_c + e;
            lb[buf][(c >> 4) * 256 + (16 * q + (c & 15)) * 4 + t] = rb[e];
        }
    };

    dv4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = dv4{0.0, 0.0, 0.0, 0.0};

    const int nk = (m + kBK - 1) / kBK;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) fetch((kc + 1) * kBK);
        double fa[2][4], fb[4][4];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const double* s = &la[buf][(2 * w + i) * 256 + lane * 4];
            const double2 x = *reinterpret_cast<const double2*>(s);
            const double2 y = *reinterpret_cast<const double2*>(s + 2);
            fa[i][0] = x.x;
            fa[i][1] = x.y;
            fa[i][2] = y.x;
            fa[i][3] = y.y;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double* s = &lb[buf][j * 256 + lane * 4];
            const double2 x = *reinterpret_cast<const double2*>(s);
            const double2 y = *reinterpret_cast<const double2*>(s + 2);
            fb[j][0] = x.x;
            fb[j][1] = x.y;
            fb[j][2] = y.x;
            fb[j][3] = y.y;
        }
        // step t contracts k = 4q + t over the lane groups q
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][t], fb[j][t], acc[i][j], 0, 0, 0);
        if (kc + 1 < nk) stash(buf ^ 1);
        __syncthreads();
    }

    // item v of lane l = 16q + c is row q + 4v, column c of its 16 x 16 output tile
    const int q = lane >> 4, c = lane & 15;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + (2 * w + i) * 16 + q + 4 * v;
            if (row >= B) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = c0 + j * 16 + c;
                if (col < n) I[row * n + col] = acc[i][j][v];
            }
        }
}

}  // namespace

hipError_t xbk_launch_transfer_apply(int B, int m, int n, const double* V, const double* T, double* I,
                                     hipStream_t s)
{
    if (B < 1 || m < 1 || n < 1 || !V || !T || !I) return hipErrorInvalidValue;
    const int64_t rp = ((int64_t)B + kBM - 1) / kBM, ct = ((int64_t)n + kBN - 1) / kBN;
    if (rp * ct > INT_MAX) return hipErrorInvalidValue;
    const int xcd_rows = rp % 8 == 0 ? (int)(rp / 8) : 0;
    const bool vec = m % 2 == 0 && n % 2 == 0 && reinterpret_cast<uintptr_t>(V) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(T) % 16 == 0;
    const dim3 grid((unsigned)(rp * ct)), block(kThreads);
    if (vec)
        hipLaunchKernelGGL(transfer_apply_kernel<true>, grid, block, 0, s, V, T, I, B, m, n, (int)ct,
                           xcd_rows);
    else
        hipLaunchKernelGGL(transfer_apply_kernel<false>, grid, block, 0, s, V, T, I, B, m, n, (int)ct,
                           xcd_rows);
    return hipGetLastError();
}

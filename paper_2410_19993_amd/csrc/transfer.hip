// Float64 matrix-core kernels of the transfer-matrix shortcut.  The crossbar is
// a linear network: the nodal system of Sec. II.A has a right-hand side that is
// linear in the word-line sources, so the output currents of any batch are the
// input voltages times the m x n matrix T of output currents per unit input.
// This file holds the product I = V T (below) and, further down, the block
// products and row reduction that build T from the factorization.
//
// Tiling (gfx950, wave64): a workgroup of 8 waves owns a 128 x 64 block of I
// and walks the contraction index k in chunks of 32.  Each chunk of V
// (128 x 32) and of T (32 x 64) is staged in LDS in matrix-core operand order:
// 16 x 16 tiles, lane l = 16q + r holding the four values k = 4q + t,
// t = 0..3, so every lane fetches its operands for four v_mfma_f64_16x16x4f64
// steps with two 16-byte LDS loads.  Thread g fills operand slot g, so a wave
// writes LDS contiguously (a row-major thread mapping is 8-way bank-conflicted
// here and costs about 30% of the kernel's time).  The waves form a 4 x 2
// grid, each computing a 32 x 32 block (2 x 2 output tiles).  Chunks are loaded
// from global memory into registers two ahead of the one the matrix cores are
// working on and written to the other of two LDS buffers: one barrier per chunk.
//
// XCD-aware launch: workgroups are dealt to the 8 XCDs round-robin.  When the
// row panels divide by 8, each XCD gets a contiguous range of row panels with
// all their column tiles, so one XCD reads each panel of V from HBM and T,
// which every workgroup reads, stays in each XCD's L2.
#include <climits>
#include <cstdint>
#include <type_traits>

#include "common.h"
#include "transfer.h"

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

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

// Block shape: BM x BN outputs, contraction chunks of BK, WM x WN waves each owning
// (BM / WM) x (BN / WN) outputs.
template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct Tiling {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
    static constexpr int kThreads = 64 * WM * WN;
    static constexpr int TI = BM / WM / 16, TJ = BN / WN / 16;   // output tiles per wave
    static constexpr int KS = BK / 16;                            // 16-deep sub-chunks per chunk
    static constexpr int GA = BM * BK / 4 / kThreads;             // 4-wide V pieces per thread
    static constexpr int GB = BN * BK / 4 / kThreads;             // 4-wide T pieces per thread
    static constexpr int LA = BM * BK, LB = BN * BK;              // doubles per LDS stage
    static_assert(TI >= 1 && TJ >= 1 && BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tiles");
    static_assert(BK % 16 == 0 && GA >= 1 && GB >= 1, "chunk");
    static_assert(GA * kThreads * 4 == BM * BK && GB * kThreads * 4 == BN * BK, "pieces");
};

// VEC: m even and V 16-byte aligned, so every 4-wide piece of a V row starts 16-byte aligned.
// LDS stage layout (both operands): [16-row tile][16-deep sub-chunk][lane][t].
template <class C, bool VEC>
__global__ __launch_bounds__(C::kThreads) void transfer_apply_kernel(
    const double* __restrict__ V, const double* __restrict__ T, double* __restrict__ I,
    int B, int m, int n, int col_tiles, int xcd_rows)
{
    __shared__ __align__(16) double la[2][C::LA];
    __shared__ __align__(16) double lb[2][C::LB];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wi = w / C::WN, wj = w % C::WN;
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
    const int64_t r0 = (int64_t)rp * C::BM;
    const int c0 = ct * C::BN;

    // Thread g fills LDS slot g of each operand (4 doubles at 32 g bytes, so the stores are
    // contiguous across a wave).  Slot g is lane l = g % 64 (l = 16q + r) of 16 x 16 operand
    // tile g / 64 = (tile, sub-chunk ks): V row 16 tile + r, k = 16 ks + 4q + t; T column
    // 16 tile + r, the same k.  A V slot is four consecutive doubles of one row; a T slot is
    // four doubles of one column.
    int a_k[C::GA];
    bool a_ok[C::GA];
    const double* a_src[C::GA];
#pragma unroll
    for (int e = 0; e < C::GA; ++e) {
        const int g = tid + C::kThreads * e, rest = g >> 6;
        const int row = 16 * (rest / C::KS) + (g & 15);
        a_k[e] = 16 * (rest % C::KS) + 4 * ((g >> 4) & 3);
        a_ok[e] = r0 + row < B;
        a_src[e] = V + (a_ok[e] ? (r0 + row) * (int64_t)m : 0) + a_k[e];
    }
    int b_k[C::GB];
    bool b_ok[C::GB];
    const double* b_src[C::GB];
#pragma unroll
    for (int e = 0; e < C::GB; ++e) {
        const int g = tid + C::kThreads * e, rest = g >> 6;
        const int col = c0 + 16 * (rest / C::KS) + (g & 15);
        b_k[e] = 16 * (rest % C::KS) + 4 * ((g >> 4) & 3);
        b_ok[e] = col < n;
        b_src[e] = T + (b_ok[e] ? col : 0);
    }

    double ra[2][C::GA][4], rb[2][C::GB][4];                  // two chunks in flight
    auto fetch = [&](int k0, auto set) {
#pragma unroll
        for (int e = 0; e < C::GA; ++e)
            load4<VEC>(a_src[e] + k0, a_ok[e] ? clamp4(m - (k0 + a_k[e])) : 0, ra[set][e]);
#pragma unroll
        for (int e = 0; e < C::GB; ++e) {
            const int k = k0 + b_k[e];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                rb[set][e][t] = (b_ok[e] && k + t < m) ? b_src[e][(int64_t)(k + t) * n] : 0.0;
        }
    };
    auto put = [](double* d, const double (&x)[4]) {
        *reinterpret_cast<double2*>(d) = double2{x[0], x[1]};
        *reinterpret_cast<double2*>(d + 2) = double2{x[2], x[3]};
    };
    auto stash = [&](int buf, auto set) {
#pragma unroll
        for (int e = 0; e < C::GA; ++e) put(&la[buf][(tid + C::kThreads * e) * 4], ra[set][e]);
#pragma unroll
        for (int e = 0; e < C::GB; ++e) put(&lb[buf][(tid + C::kThreads * e) * 4], rb[set][e]);
    };

    dv4 acc[C::TI][C::TJ];
#pragma unroll
    for (int i = 0; i < C::TI; ++i)
#pragma unroll
        for (int j = 0; j < C::TJ; ++j) acc[i][j] = dv4{0.0, 0.0, 0.0, 0.0};

    auto compute = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < C::KS; ++ks) {
            double fa[C::TI][4], fb[C::TJ][4];
#pragma unroll
            for (int i = 0; i < C::TI; ++i) {
                const double* s = &la[buf][((wi * C::TI + i) * C::KS + ks) * 256 + lane * 4];
                const double2 x = *reinterpret_cast<const double2*>(s);
                const double2 y = *reinterpret_cast<const double2*>(s + 2);
                fa[i][0] = x.x;
                fa[i][1] = x.y;
                fa[i][2] = y.x;
                fa[i][3] = y.y;
            }
#pragma unroll
            for (int j = 0; j < C::TJ; ++j) {
                const double* s = &lb[buf][((wj * C::TJ + j) * C::KS + ks) * 256 + lane * 4];
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
                for (int i = 0; i < C::TI; ++i)
#pragma unroll
                    for (int j = 0; j < C::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][t], fb[j][t], acc[i][j], 0, 0, 0);
        }
    };

    // register set s holds the chunk kc + 1 while the chunk kc + 2 loads into the other
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    const int nk = (m + C::BK - 1) / C::BK;
    fetch(0, S0{});
    stash(0, S0{});
    if (nk > 1) fetch(C::BK, S1{});
    __syncthreads();
    auto step = [&](int kc, auto cur, auto nxt) {
        if (kc + 2 < nk) fetch((kc + 2) * C::BK, cur);
        compute(kc & 1);
        if (kc + 1 < nk) stash((kc & 1) ^ 1, nxt);
        __syncthreads();
    };
    for (int kc = 0; kc < nk; kc += 2) {
        step(kc, S0{}, S1{});
        if (kc + 1 < nk) step(kc + 1, S1{}, S0{});
    }

    // item v of lane l = 16q + c is row q + 4v, column c of its 16 x 16 output tile
    const int q = lane >> 4, c = lane & 15;
#pragma unroll
    for (int i = 0; i < C::TI; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + (wi * C::TI + i) * 16 + q + 4 * v;
            if (row >= B) continue;
#pragma unroll
            for (int j = 0; j < C::TJ; ++j) {
                const int col = c0 + (wj * C::TJ + j) * 16 + c;
                if (col < n) I[row * n + col] = acc[i][j][v];
            }
        }
}

template <class C>
hipError_t launch_tiling(int B, int m, int n, const double* V, const double* T, double* I, hipStream_t s)
{
    const int64_t rp = ((int64_t)B + C::BM - 1) / C::BM, ct = ((int64_t)n + C::BN - 1) / C::BN;
    if (rp * ct > INT_MAX) return hipErrorInvalidValue;
    const int xcd_rows = rp % 8 == 0 ? (int)(rp / 8) : 0;
    const bool vec = m % 2 == 0 && reinterpret_cast<uintptr_t>(V) % 16 == 0;
    const dim3 grid((unsigned)(rp * ct)), block(C::kThreads);
    if (vec)
        hipLaunchKernelGGL((transfer_apply_kernel<C, true>), grid, block, 0, s, V, T, I, B, m, n, (int)ct,
                           xcd_rows);
    else
        hipLaunchKernelGGL((transfer_apply_kernel<C, false>), grid, block, 0, s, V, T, I, B, m, n, (int)ct,
                           xcd_rows);
    return hipGetLastError();
}

using ApplyTiling = Tiling<128, 64, 32, 4, 2>;

// ---------------------------------------------------------------------------
// Products of FRG blocks for building T from the factorization.  A workgroup of 4
// waves owns a 32 x 32 output block (2 x 2 tiles); wave w covers a quarter of the
// contraction for all four tiles (so each operand tile is read once per workgroup),
// and the partial tiles are summed through LDS.  With the A slot of the matrix core
// fed from the tile of B and the B slot from the tile of A, item v of lane l is
// element (l % 16, kidx(l / 16, v)) of the tile of A B^T: partials and output are in
// FRG order with no shuffle.
struct FrgProductArgs {
    XbkFrgJob job[2];
    int n_p;
    double alpha;
};

__global__ __launch_bounds__(256) void frg_product_kernel(FrgProductArgs a)
{
    using F = xbk::Frag<double>;
    __shared__ __align__(16) double part[4][4][256];      // [wave][output tile][slot]
    const int TP = a.n_p / 32, T2 = TP * TP, KT = a.n_p / 16, KQ = KT / 4;
    const int jb = blockIdx.x / T2, t2 = blockIdx.x % T2;
    const XbkFrgJob J = a.job[jb];
    int tr2, tc2;
    if (TP % 4 == 0) {
        // XCD b % 8 owns a quarter of the block rows and half of the block columns
        const int xcd = t2 & 7, local = t2 >> 3;
        tr2 = (xcd >> 1) * (TP / 4) + local / (TP / 2);
        tc2 = (xcd & 1) * (TP / 2) + local % (TP / 2);
    } else {
        tr2 = t2 / TP;
        tc2 = t2 % TP;
    }
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    // tiles (2 tr2 + i, k) of A and (2 tc2 + j, k) of B for k in this wave's quarter
    const double* pa = J.A + ((int64_t)(2 * tr2) * KT + w * KQ) * 256;
    const double* pb = J.B + ((int64_t)(2 * tc2) * KT + w * KQ) * 256;
    const int64_t row_step = (int64_t)KT * 256;
    auto frag = [&](const double* t, double (&x)[4]) {
        const double2 lo = *reinterpret_cast<const double2*>(t + 2 * l);
        const double2 hi = *reinterpret_cast<const double2*>(t + 128 + 2 * l);
        x[0] = lo.x;
        x[1] = lo.y;
        x[2] = hi.x;
        x[3] = hi.y;
    };
    F::acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = F::acc_t{0.0, 0.0, 0.0, 0.0};
    double fa[2][2][4], fb[2][2][4];                        // [buffer][tile][t]
    auto load = [&](int k, int buf) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            frag(pa + i * row_step + k * 256, fa[buf][i]);
            frag(pb + i * row_step + k * 256, fb[buf][i]);
        }
    };
    auto step = [&](int buf) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = F::mma(fb[buf][j][t], fa[buf][i][t], acc[i][j]);
    };
    load(0, 0);
    for (int k = 0; k < KQ; k += 2) {
        if (k + 1 < KQ) load(k + 1, 1);
        step(0);
        if (k + 1 < KQ) {
            if (k + 2 < KQ) load(k + 2, 0);
            step(1);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) part[w][2 * i + j][xbk::frg_slot<double>(l, v)] = acc[i][j][v];
    __syncthreads();
    // wave w sums output tile (i, j) = (w >> 1, w & 1) over the four quarters
    const int tr = 2 * tr2 + (w >> 1), tc = 2 * tc2 + (w & 1);
    const int64_t o = ((int64_t)tr * KT + tc) * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int e = xbk::frg_slot<double>(l, v);
        const double sum = ((part[0][w][e] + part[1][w][e]) + part[2][w][e]) + part[3][w][e];
        const double c = J.C ? J.C[o + e] : 0.0;
        J.out[o + e] = a.alpha * sum + c;
    }
}

// T[i][j] = g_sense sum_{k < n} W_i[j][k] c_i[k]: workgroup (i, 64-row group), lane j,
// the k sum in order over the FRG positions of row j
__global__ __launch_bounds__(64) void transfer_rows_kernel(int m, int n, int n_p, const double* __restrict__ W,
                                                           const double* __restrict__ c, double g_sense,
                                                           double* __restrict__ T)
{
    const int i = blockIdx.x / (n_p / 64), j = (blockIdx.x % (n_p / 64)) * 64 + threadIdx.x;
    if (i >= m || j >= n) return;
    const double* Wi = W + (int64_t)i * n_p * n_p;
    const double* ci = c + (int64_t)i * n_p;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += Wi[xbk::frg<double>(j, k, n_p)] * ci[k];
    T[(int64_t)i * n + j] = g_sense * s;
}

}  // namespace

hipError_t xbk_launch_frg_products(const XbkFrgJob* jobs, int njobs, int n_p, double alpha, hipStream_t s)
{
    if (njobs < 1 || njobs > 2 || n_p < 64 || n_p % 64 != 0) return hipErrorInvalidValue;
    FrgProductArgs a{};
    for (int k = 0; k < njobs; ++k) {
        if (!jobs[k].A || !jobs[k].B || !jobs[k].out) return hipErrorInvalidValue;
        a.job[k] = jobs[k];
    }
    a.n_p = n_p;
    a.alpha = alpha;
    const int TP = n_p / 32;
    hipLaunchKernelGGL(frg_product_kernel, dim3(njobs * TP * TP), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t xbk_launch_transfer_rows(int m, int n, int n_p, const double* W, const double* c, double g_sense,
                                    double* T, hipStream_t s)
{
    if (m < 1 || n < 1 || n > n_p || n_p % 64 != 0 || !W || !c || !T) return hipErrorInvalidValue;
    const int64_t grid = (int64_t)m * (n_p / 64);
    if (grid > INT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(transfer_rows_kernel, dim3((unsigned)grid), dim3(64), 0, s, m, n, n_p, W, c, g_sense, T);
    return hipGetLastError();
}

hipError_t xbk_launch_transfer_apply(int B, int m, int n, const double* V, const double* T, double* I,
                                     hipStream_t s)
{
    if (B < 1 || m < 1 || n < 1 || !V || !T || !I) return hipErrorInvalidValue;
    return launch_tiling<ApplyTiling>(B, m, n, V, T, I, s);
}

// The surrogate's 3 x 3 convolutions on the bfloat16 matrix cores
// (v_mfma_f32_16x16x32_bf16: bfloat16 operands, float32 accumulation), for the
// same layouts and results as the float32 kernels of surrogate.hip: activations and
// gradients stay float32 in memory and are rounded to bfloat16 (nearest, ties to
// even) when a workgroup stages them; the weights are rounded when loaded.
//
// Matrix-core layout (lane l, item i; checked on gfx950 with integer operands):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + i], i = 0..7
//   B (32 x 16): lane l holds B[8 (l / 16) + i][l % 16]
//   D (16 x 16): lane l item v holds D[4 (l / 16) + v][l % 16]
//
// Forward and input gradient are one implicit GEMM: a workgroup of four waves owns a
// 16 x 16 tile of crosspoints of one sample (wave w: rows 4w .. 4w+3, a 16-crosspoint
// strip each), with the input tile and its halo staged in LDS as [18 x 18 positions]
// x [channels] bfloat16, so that the eight channels a lane needs for one tap are one
// 16-byte read.  The contraction runs over (tap, 8-channel chunk) pairs, four pairs
// (32 = K) per matrix-core step; the weights' B fragments stay in registers for the
// whole (persistent) workgroup.  The input gradient is the forward convolution of the
// masked output gradient with the weights transposed over channels and flipped over
// taps: gx[c](p, q) = sum_{o, t'} w[o][c][8 - t'] g[o](p + dy' - 1, q + dx' - 1).
//
// Weight gradient: for each tap t, gw_t[o][c] = sum over crosspoints of g[o] and the
// input shifted by t: an O x C x (crosspoints) GEMM per tap.  A workgroup takes 16 x 16
// crosspoint tiles in turn (positions p * 16 + q are the contraction index), with g as
// [O] x [256 positions] and three column-shifted copies of the input as
// [3][C][18 rows][16 columns] in LDS, so that every operand read is an aligned 16-byte
// read.  Wave (mt, nt) accumulates the 16 x 16 block (mt, nt) of all nine taps.
// Per-workgroup partial sums are added in a fixed order by sg_reduce_parts_kernel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "xbar.h"

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float fv4_t __attribute__((ext_vector_type(4)));

namespace {

constexpr int kT = 16;            // crosspoint tile edge
constexpr int kH = kT + 2;        // with the halo
constexpr int kWgParts = 512;     // weight-gradient workgroups (partial sums), as the float32 pass

__device__ __forceinline__ fv4_t mma(const bf8_t& a, const bf8_t& b, const fv4_t& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bool inside(int p, int q, int H, int W) { return p >= 0 && p < H && q >= 0 && q < W; }

// Implicit-GEMM 3 x 3 convolution, CP = input channels rounded up to 8 (a multiple of 8
// up to 32), NT = output-channel tiles of 16 (1 or 2).  BWD: input gradient (the input
// is the output gradient, masked by [mask_in > 0]; the output is multiplied by
// [mask_out > 0]); else forward (bias, then ReLU when relu != 0).
template <int CP, int NT, bool BWD>
__global__ __launch_bounds__(256) void sg_conv_mfma_kernel(int B, int H, int W, int Cin, int Cout, int relu,
                                                           const float* __restrict__ x,
                                                           const float* __restrict__ mask_in,
                                                           const float* __restrict__ w,
                                                           const float* __restrict__ bias,
                                                           const float* __restrict__ mask_out, float* __restrict__ y)
{
    constexpr int NCH = CP / 8;                 // 8-channel chunks
    constexpr int P = 9 * NCH;                  // (tap, chunk) pairs
    constexpr int S = (P + 3) / 4;              // matrix-core steps (K = 32 each)
    constexpr int PS = CP + 8;                  // LDS elements per position (16-byte aligned, padded)
    __shared__ __align__(16) __bf16 xt[kH * kH * PS];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, g = l >> 4, c16 = l & 15;
    // B fragments: lane l, output channel nt*16 + l%16, pair 4 s + l/16 (8 input channels)
    bf8_t wf[S][NT];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int j = 4 * s + g, oc = nt * 16 + c16;
            const int t = j / NCH, cc = j % NCH;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int ic = 8 * cc + i;
                float v = 0.0f;
                if (j < P && oc < Cout && ic < Cin)
                    v = BWD ? w[((int64_t)ic * Cout + oc) * 9 + (8 - t)] : w[((int64_t)oc * Cin + ic) * 9 + t];
                wf[s][nt][i] = (__bf16)v;
            }
        }
    float bo[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int oc = nt * 16 + c16;
        bo[nt] = (!BWD && oc < Cout) ? bias[oc] : 0.0f;
    }
    const int th = (H + kT - 1) / kT, tw = (W + kT - 1) / kT;
    const int tiles = B * th * tw;
    const int64_t hw = (int64_t)H * W;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int b = tile / (th * tw), r = tile % (th * tw);
        const int p0 = (r / tw) * kT, q0 = (r % tw) * kT;
        __syncthreads();                                  // the previous tile's reads are done
        // stage the input tile with its halo: [position][channel], bfloat16
        const float* xb = x + (int64_t)b * Cin * hw;
        const float* mb = mask_in ? mask_in + (int64_t)b * Cin * hw : nullptr;
        for (int e = threadIdx.x; e < CP * kH * kH; e += 256) {
            const int c = e / (kH * kH), pos = e % (kH * kH);
            const int pp = p0 + pos / kH - 1, qq = q0 + pos % kH - 1;
            float v = 0.0f;
            if (c < Cin && inside(pp, qq, H, W)) {
                const int64_t o = c * hw + (int64_t)pp * W + qq;
                v = xb[o];
                if (mb && !(mb[o] > 0.0f)) v = 0.0f;
            }
            xt[pos * PS + c] = (__bf16)v;
        }
        __syncthreads();
        fv4_t acc[4][NT];
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[st][nt] = fv4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = 4 * s + g;
            const int t = j / NCH, cc = j % NCH;
            const int dy = t / 3, dx = t % 3;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int pl = 4 * wv + st;               // tile row of this strip
                bf8_t a;
                if (j < P)
                    a = *reinterpret_cast<const bf8_t*>(xt + ((pl + dy) * kH + c16 + dx) * PS + 8 * cc);
                else
#pragma unroll
                    for (int i = 0; i < 8; ++i) a[i] = (__bf16)0.0f;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[st][nt] = mma(a, wf[s][nt], acc[st][nt]);
            }
        }
        // D lane l item v: crosspoint 4 (l / 16) + v of the strip, output channel l % 16
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int p = p0 + 4 * wv + st;
            if (p >= H) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int oc = nt * 16 + c16;
                if (oc >= Cout) continue;
                float* yo = y + ((int64_t)b * Cout + oc) * hw + (int64_t)p * W;
                const float* mo = mask_out ? mask_out + ((int64_t)b * Cout + oc) * hw + (int64_t)p * W : nullptr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = q0 + 4 * g + v;
                    if (q >= W) continue;
                    float val = acc[st][nt][v];
                    if (!BWD) {
                        val += bo[nt];
                        if (relu) val = fmaxf(val, 0.0f);
                    } else if (mo && !(mo[q] > 0.0f)) {
                        val = 0.0f;
                    }
                    yo[q] = val;
                }
            }
        }
    }
}

// Weight and bias gradient partial sums of one workgroup: NO, NC = tiles of 16 output
// and input channels (1 or 2 each).  part: [gridDim.x][O C 9 + O], laid out as the
// weights [o][c][tap], then the biases.
template <int NO, int NC>
__global__ __launch_bounds__(256) void sg_wgrad_mfma_kernel(int B, int H, int W, int C, int O,
                                                            const float* __restrict__ x,
                                                            const float* __restrict__ gy,
                                                            const float* __restrict__ ymask,
                                                            float* __restrict__ part)
{
    // LDS strides: 16-byte reads by 8 lanes of consecutive rows (g) or channels (x) hit
    // distinct banks when the stride is an odd multiple of 4 words
    constexpr int GS = kT * kT + 8;               // elements per g row: 132 words
    constexpr int RS = kT;                        // elements per x row (16-byte aligned)
    constexpr int CS = kH * RS + 8;               // elements per x channel: 148 words
    constexpr int CR = 16 * NC;                   // input channels staged
    __shared__ __align__(16) __bf16 gs[16 * NO * GS];
    __shared__ __align__(16) __bf16 xs[3 * CR * CS];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, g = l >> 4, c16 = l & 15;
    const int mt = wv >> 1, nt = wv & 1;
    const bool active = mt < NO && nt < NC;
    fv4_t acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = fv4_t{0.0f, 0.0f, 0.0f, 0.0f};
    float accb = 0.0f;
    const int th = (H + kT - 1) / kT, tw = (W + kT - 1) / kT;
    const int tiles = B * th * tw;
    const int64_t hw = (int64_t)H * W;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int b = tile / (th * tw), r = tile % (th * tw);
        const int p0 = (r / tw) * kT, q0 = (r % tw) * kT;
        __syncthreads();
        const float* gb = gy + (int64_t)b * O * hw;
        const float* mb = ymask ? ymask + (int64_t)b * O * hw : nullptr;
        for (int e = threadIdx.x; e < 16 * NO * kT * kT; e += 256) {
            const int o = e / (kT * kT), pos = e % (kT * kT);
            const int pp = p0 + pos / kT, qq = q0 + pos % kT;
            float v = 0.0f;
            if (o < O && pp < H && qq < W) {
                const int64_t off = o * hw + (int64_t)pp * W + qq;
                v = gb[off];
                if (mb && !(mb[off] > 0.0f)) v = 0.0f;
            }
            gs[o * GS + pos] = (__bf16)v;
        }
        // three copies of the input tile, copy dx holding columns q0 + dx - 1 .. + 15
        const float* xb = x + (int64_t)b * C * hw;
        for (int e = threadIdx.x; e < CR * kH * kH; e += 256) {
            const int c = e / (kH * kH), pos = e % (kH * kH);
            const int rr = pos / kH, cq = pos % kH;            // halo row 0..17, halo column 0..17
            const int pp = p0 + rr - 1, qq = q0 + cq - 1;
            const __bf16 v = (__bf16)((c < C && inside(pp, qq, H, W)) ? xb[c * hw + (int64_t)pp * W + qq] : 0.0f);
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int col = cq - dx;                       // column of copy dx
                if (col >= 0 && col < kT) xs[(dx * CR + c) * CS + rr * RS + col] = v;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll 2
            for (int s = 0; s < kT * kT / 32; ++s) {
                // A: g rows mt*16 + l%16, positions 32 s + 8 (l/16) .. + 7
                const bf8_t a = *reinterpret_cast<const bf8_t*>(gs + (mt * 16 + c16) * GS + 32 * s + 8 * g);
                const int pos = 32 * s + 8 * g, p = pos / kT, q = pos % kT;
                const int c = nt * 16 + c16;
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int dy = t / 3, dx = t % 3;
                    const bf8_t bq = *reinterpret_cast<const bf8_t*>(xs + (dx * CR + c) * CS + (p + dy) * RS + q);
                    acc[t] = mma(a, bq, acc[t]);
                }
            }
        }
        if (threadIdx.x < O) {
            float sb = 0.0f;
            for (int e = 0; e < kT * kT; ++e) sb += (float)gs[threadIdx.x * GS + e];
            accb += sb;
        }
    }
    const int ne = O * C * 9;
    float* pw = part + (int64_t)blockIdx.x * (ne + O);
    if (active) {
        const int c = nt * 16 + c16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = mt * 16 + 4 * g + v;
            if (o < O && c < C)
#pragma unroll
                for (int t = 0; t < 9; ++t) pw[((int64_t)o * C + c) * 9 + t] = acc[t][v];
        }
    }
    if (threadIdx.x < O) pw[ne + threadIdx.x] = accb;
}

template <bool BWD>
hipError_t launch_conv(int B, int H, int W, int Cin, int Cout, int relu, const float* x, const float* mask_in,
                       const float* w, const float* bias, const float* mask_out, float* y, hipStream_t s)
{
    const int64_t tiles = (int64_t)B * ((H + kT - 1) / kT) * ((W + kT - 1) / kT);
    const int grid = (int)(tiles < 2048 ? tiles : 2048);
    const int cp = ((Cin + 7) / 8) * 8;
    const bool two = Cout > 16;
#define XB_CONV(CPV)                                                                                               \
    if (two)                                                                                                       \
        hipLaunchKernelGGL((sg_conv_mfma_kernel<CPV, 2, BWD>), dim3(grid), dim3(256), 0, s, B, H, W, Cin, Cout,   \
                           relu, x, mask_in, w, bias, mask_out, y);                                                 \
    else                                                                                                           \
        hipLaunchKernelGGL((sg_conv_mfma_kernel<CPV, 1, BWD>), dim3(grid), dim3(256), 0, s, B, H, W, Cin, Cout,   \
                           relu, x, mask_in, w, bias, mask_out, y);
    switch (cp) {
        case 8: XB_CONV(8) break;
        case 16: XB_CONV(16) break;
        case 24: XB_CONV(24) break;
        default: XB_CONV(32) break;
    }
#undef XB_CONV
    return hipGetLastError();
}

}  // namespace

hipError_t xbk_sg_conv_forward_bf16(int B, int H, int W, int C, int O, int relu, const float* x, const float* w,
                                    const float* bias, float* y, hipStream_t s)
{
    return launch_conv<false>(B, H, W, C, O, relu, x, nullptr, w, bias, nullptr, y, s);
}

hipError_t xbk_sg_conv_backward_data_bf16(int B, int H, int W, int C, int O, const float* gy, const float* ymask,
                                          const float* w, const float* xmask, float* gx, hipStream_t s)
{
    // the forward convolution of the masked gradient (O channels in) to C channels out
    return launch_conv<true>(B, H, W, O, C, 0, gy, ymask, w, nullptr, xmask, gx, s);
}

hipError_t xbk_sg_conv_backward_weight_bf16(int B, int H, int W, int C, int O, const float* x, const float* gy,
                                            const float* ymask, float* part, int nparts, hipStream_t s)
{
    const bool o2 = O > 16, c2 = C > 16;
    if (o2 && c2)
        hipLaunchKernelGGL((sg_wgrad_mfma_kernel<2, 2>), dim3(nparts), dim3(256), 0, s, B, H, W, C, O, x, gy, ymask, part);
    else if (o2)
        hipLaunchKernelGGL((sg_wgrad_mfma_kernel<2, 1>), dim3(nparts), dim3(256), 0, s, B, H, W, C, O, x, gy, ymask, part);
    else if (c2)
        hipLaunchKernelGGL((sg_wgrad_mfma_kernel<1, 2>), dim3(nparts), dim3(256), 0, s, B, H, W, C, O, x, gy, ymask, part);
    else
        hipLaunchKernelGGL((sg_wgrad_mfma_kernel<1, 1>), dim3(nparts), dim3(256), 0, s, B, H, W, C, O, x, gy, ymask, part);
    return hipGetLastError();
}

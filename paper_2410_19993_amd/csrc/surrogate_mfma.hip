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
// Forward and input gradient are one implicit GEMM: a persistent workgroup of four
// waves takes 8 x 32 tiles of crosspoints of one sample in turn (16 strips of 16
// crosspoints, four per wave), with the input tile and its halo staged in LDS as
// [10 x 34 positions] x [channels] bfloat16, so that the eight channels a lane needs
// for one tap are one 16-byte read.  The contraction runs over (tap, 8-channel chunk)
// pairs, four pairs (32 = K) per matrix-core step; the weights sit in LDS for the whole
// workgroup, and the next tile's input is loaded while the current one is computed.
// The input gradient is the forward convolution of the masked output gradient with the
// weights transposed over channels and flipped over taps:
// gx[c](p, q) = sum_{o, t'} w[o][c][8 - t'] g[o](p + dy' - 1, q + dx' - 1).
//
// Weight gradient: for each tap t, gw_t[o][c] = sum over crosspoints of g[o] and the
// input shifted by t: an O x C x (crosspoints) GEMM per tap.  A workgroup takes 8 x 32
// crosspoint tiles in turn (positions p * 32 + q are the contraction index), with g as
// [O] x [256 positions] and the input with its halo as [C][10 rows][40 columns] in
// LDS; the B fragments of the three column taps come from one aligned 16-byte read and
// the dword after it, shifted by 0, 1 or 2 bfloat16.  Wave (mt, nt) accumulates the
// 16 x 16 block (mt, nt) of all nine taps.  Per-workgroup partial sums are added in a
// fixed order by sg_reduce_parts_kernel.
//
// Tiles go to the XCDs in contiguous ranges (see my_tiles), and every global load of a
// staging pass is issued before the first of them is used.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "xbar.h"

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float fv4_t __attribute__((ext_vector_type(4)));

namespace {

// Tiles of 8 x 32 crosspoints: each tile row is a full 128-byte line of float32, so a
// workgroup's loads and stores move whole lines.
constexpr int kTH = 8, kTW = 32;          // tile rows and columns
constexpr int kHH = kTH + 2, kHW = kTW + 2;   // with the halo
constexpr int kSR = kTW / 16;             // 16-crosspoint strips per tile row
static_assert(kTH * kTW == 256 && kTW % 16 == 0, "256 crosspoints per tile, whole strips per row");
#ifndef XB_SG_CONV_GRID
#define XB_SG_CONV_GRID 512
#endif
// persistent workgroups of the implicit GEMM: two fit a CU (registers), so each keeps its
// weight fragments for several tiles
constexpr int kConvGrid = XB_SG_CONV_GRID;

__device__ __forceinline__ fv4_t mma(const bf8_t& a, const bf8_t& b, const fv4_t& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bool inside(int p, int q, int H, int W) { return p >= 0 && p < H && q >= 0 && q < W; }

// p[o] when ok, else 0, with the load itself unconditional (at p[0] when !ok, which
// must be readable): a load under a branch is waited for on its own, so guarded loads
// would run one memory round trip each instead of all in flight together.
__device__ __forceinline__ float ld_or0(const float* __restrict__ p, int64_t o, bool ok)
{
    const float v = p[ok ? o : 0];
    return ok ? v : 0.0f;
}

// The tiles of a persistent workgroup.  Workgroups are dispatched to the eight XCDs in
// turn (workgroup w on XCD w % 8); when the grid is a multiple of 8, each XCD takes a
// contiguous eighth of the tiles, so that neighbouring tiles, which share halo rows and
// 128-byte lines, are fetched into the same L2 instead of into up to eight.
struct TileRange {
    int first, end, step;
};
__device__ __forceinline__ TileRange my_tiles(int tiles)
{
    if (gridDim.x % 8 != 0) return {(int)blockIdx.x, tiles, (int)gridDim.x};
    const int xcd = blockIdx.x & 7;
    const int lo = (int)((int64_t)xcd * tiles / 8), hi = (int)((int64_t)(xcd + 1) * tiles / 8);
    return {lo + (int)(blockIdx.x >> 3), hi, (int)(gridDim.x >> 3)};
}

__device__ __forceinline__ bf8_t pack8(const float (&v)[8])
{
    bf8_t r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = (__bf16)v[i];
    return r;
}

// One thread's share of an input tile of crosspoints (p0 .., q0 ..) with its
// one-crosspoint halo, for the LDS layout [18 x 18 positions][CP channels] bfloat16.
// Item r = (8-channel chunk, position), positions running fastest over the lanes.  The
// values are the raw loads (from clamped addresses): which of them are real is decided
// when they are stored, so that the loads of the next tile stay in flight, unwaited,
// while the current tile is computed.
template <int CP, bool MIN>
struct Halo {
    static constexpr int NPOS = kHH * kHW;
    static constexpr int ITEMS = NPOS * (CP / 8);
    static constexpr int ROUNDS = (ITEMS + 255) / 256;
    float v[ROUNDS][8];
    float m[MIN ? ROUNDS : 1][8];      // the input mask (MIN)

    // valid channel count of item r's chunk, -1 when the item is outside the tile or map
    __device__ __forceinline__ static int item(int r, int Cin, int H, int W, int64_t hw, int p0, int q0, int& pos,
                                               int& cc, int64_t& off)
    {
        const int e = r * 256 + threadIdx.x;
        cc = e / NPOS;
        pos = e - cc * NPOS;
        const int pp = p0 + pos / kHW - 1, qq = q0 + pos % kHW - 1;
        const bool ok = e < ITEMS && inside(pp, qq, H, W);
        off = ok ? (int64_t)(8 * cc) * hw + (int64_t)pp * W + qq : 0;
        return ok ? Cin - 8 * cc : -1;
    }

    __device__ __forceinline__ void load(const float* __restrict__ xb, const float* __restrict__ mb, int Cin, int H,
                                         int W, int64_t hw, int p0, int q0)
    {
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            int pos, cc;
            int64_t off;
            const int nc = item(r, Cin, H, W, hw, p0, q0, pos, cc, off);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int64_t o = i < nc ? off + i * hw : 0;
                v[r][i] = xb[o];
                if constexpr (MIN) m[r][i] = mb[o];
            }
        }
    }

    __device__ __forceinline__ void store(__bf16* __restrict__ xt, int Cin, int H, int W, int64_t hw, int p0,
                                          int q0) const
    {
        constexpr int PS = CP + 8;
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            int pos, cc;
            int64_t off;
            const int nc = item(r, Cin, H, W, hw, p0, q0, pos, cc, off);
            float t[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                bool keep = i < nc;
                if constexpr (MIN) keep = keep && m[r][i] > 0.0f;
                t[i] = keep ? v[r][i] : 0.0f;
            }
            if (r * 256 + threadIdx.x < ITEMS) *reinterpret_cast<bf8_t*>(xt + pos * PS + 8 * cc) = pack8(t);
        }
    }
};

// The same share with 16-byte loads, for W % 4 == 0 and 16-byte aligned rows: interior
// item (4-channel quad, halo row, group of 4 columns) loads four crosspoints of each of
// four channels (a wave reads eight full 128-byte lines per instruction) and writes four
// positions of 4 channels; edge item (8-channel chunk, halo row, left or right halo
// column) loads one crosspoint of eight.  Four times fewer load instructions than one
// crosspoint per lane, which keeps the address units from being the bottleneck.
template <int CP>
struct HaloVec {
    static constexpr int NQ = CP / 4;                           // 4-channel quads
    static constexpr int NG = kTW / 4;                          // column groups per row
    static constexpr int IN_ITEMS = NQ * kHH * NG;
    static constexpr int IN_ROUNDS = (IN_ITEMS + 255) / 256;
    static constexpr int ED_ITEMS = (CP / 8) * kHH * 2;
    static constexpr int ED_ROUNDS = (ED_ITEMS + 255) / 256;
    fv4_t v[IN_ROUNDS][4];
    float ve[ED_ROUNDS][8];

    __device__ __forceinline__ static void in_item(int r, int& cq, int& rr, int& grp)
    {
        const int e = r * 256 + threadIdx.x;
        grp = e % NG;
        rr = (e / NG) % kHH;
        cq = e / (NG * kHH);
    }
    __device__ __forceinline__ static void ed_item(int r, int& cc, int& rr, int& side)
    {
        const int e = r * 256 + threadIdx.x;
        side = e & 1;
        rr = (e >> 1) % kHH;
        cc = (e >> 1) / kHH;
    }

    __device__ __forceinline__ void load(const float* __restrict__ xb, const float*, int Cin, int H, int W,
                                         int64_t hw, int p0, int q0)
    {
#pragma unroll
        for (int r = 0; r < IN_ROUNDS; ++r) {
            int cq, rr, grp;
            in_item(r, cq, rr, grp);
            const int pp = p0 + rr - 1, qq = q0 + 4 * grp;
            const bool ok = r * 256 + (int)threadIdx.x < IN_ITEMS && pp >= 0 && pp < H && qq < W;
            const int64_t off = (int64_t)(4 * cq) * hw + (int64_t)pp * W + qq;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                v[r][i] = *reinterpret_cast<const fv4_t*>(xb + (ok && 4 * cq + i < Cin ? off + i * hw : 0));
        }
#pragma unroll
        for (int r = 0; r < ED_ROUNDS; ++r) {
            int cc, rr, side;
            ed_item(r, cc, rr, side);
            const int pp = p0 + rr - 1, qq = side ? q0 + kTW : q0 - 1;
            const bool ok = r * 256 + (int)threadIdx.x < ED_ITEMS && inside(pp, qq, H, W);
            const int64_t off = (int64_t)(8 * cc) * hw + (int64_t)pp * W + qq;
#pragma unroll
            for (int i = 0; i < 8; ++i) ve[r][i] = xb[ok && 8 * cc + i < Cin ? off + i * hw : 0];
        }
    }

    __device__ __forceinline__ void store(__bf16* __restrict__ xt, int Cin, int H, int W, int64_t, int p0,
                                          int q0) const
    {
        typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
        constexpr int PS = CP + 8;
#pragma unroll
        for (int r = 0; r < IN_ROUNDS; ++r) {
            int cq, rr, grp;
            in_item(r, cq, rr, grp);
            if (r * 256 + (int)threadIdx.x >= IN_ITEMS) continue;
            const int pp = p0 + rr - 1, qq = q0 + 4 * grp;
            const bool ok = pp >= 0 && pp < H && qq < W;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                bf4_t t;
#pragma unroll
                for (int i = 0; i < 4; ++i) t[i] = (__bf16)((ok && 4 * cq + i < Cin) ? v[r][i][k] : 0.0f);
                *reinterpret_cast<bf4_t*>(xt + (rr * kHW + 1 + 4 * grp + k) * PS + 4 * cq) = t;
            }
        }
#pragma unroll
        for (int r = 0; r < ED_ROUNDS; ++r) {
            int cc, rr, side;
            ed_item(r, cc, rr, side);
            if (r * 256 + (int)threadIdx.x >= ED_ITEMS) continue;
            const int pp = p0 + rr - 1, qq = side ? q0 + kTW : q0 - 1;
            const bool ok = inside(pp, qq, H, W);
            float t[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) t[i] = (ok && 8 * cc + i < Cin) ? ve[r][i] : 0.0f;
            *reinterpret_cast<bf8_t*>(xt + (rr * kHW + (side ? kHW - 1 : 0)) * PS + 8 * cc) = pack8(t);
        }
    }
};

// Implicit-GEMM 3 x 3 convolution, CP = input channels rounded up to 8 (a multiple of 8
// up to 32), NT = output-channel tiles of 16 (1 or 2).  BWD: input gradient (the input
// is the output gradient, masked by [mask_in > 0] when MIN; the output is multiplied by
// [mask_out > 0]); else forward (bias, then ReLU when relu != 0).  VEC: W % 4 == 0 and
// every array 16-byte aligned (16-byte loads and stores).
template <int CP, int NT, bool BWD, bool MIN, bool VEC>
__global__ __launch_bounds__(256, 2) void sg_conv_mfma_kernel(int B, int H, int W, int Cin, int Cout, int relu,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ mask_in,
                                                              const float* __restrict__ w,
                                                              const float* __restrict__ bias,
                                                              const float* __restrict__ mask_out,
                                                              float* __restrict__ y)
{
    constexpr int NCH = CP / 8;                 // 8-channel chunks
    constexpr int P = 9 * NCH;                  // (tap, chunk) pairs
    constexpr int S = (P + 3) / 4;              // matrix-core steps (K = 32 each)
    constexpr int PS = CP + 8;                  // LDS elements per position (16-byte aligned, padded)
    constexpr int OC = 16 * NT;
    __shared__ __align__(16) __bf16 xt[kHH * kHW * PS];
    // the weights, rounded to bfloat16, as [tap][OC output channels][PS input channels]
    // (zero padded): lane l's B fragment for pair j = (tap, chunk) and output channel oc
    // is one 16-byte read, and eight lanes of consecutive oc hit distinct banks
    __shared__ __align__(16) __bf16 wl[9 * OC * PS];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, g = l >> 4, c16 = l & 15;
    for (int e = threadIdx.x; e < 9 * OC * PS; e += 256) wl[e] = (__bf16)0.0f;
    __syncthreads();
    {
        const int nw = Cin * Cout * 9;
#pragma unroll 8
        for (int e = threadIdx.x; e < nw; e += 256) {
            const float v = w[e];
            const int tap = e % 9, r = e / 9;
            // forward: w[oc][ic][tap]; input gradient: w[ic][oc][8 - tap] (ic = the
            // convolution's input channel, an output channel of the layer)
            const int oc = BWD ? r % Cout : r / Cin, ic = BWD ? r / Cout : r % Cin, t = BWD ? 8 - tap : tap;
            wl[(t * OC + oc) * PS + ic] = (__bf16)v;
        }
    }
    float bo[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int oc = nt * 16 + c16;
        if constexpr (BWD)
            bo[nt] = 0.0f;
        else
            bo[nt] = ld_or0(bias, oc, oc < Cout);
    }
    const int th = (H + kTH - 1) / kTH, tw = (W + kTW - 1) / kTW;
    const int tiles = B * th * tw;
    const int64_t hw = (int64_t)H * W;
    // rows of 16-byte aligned float4s
    constexpr bool vec = VEC;
    const TileRange tr = my_tiles(tiles);
    // 16-byte loads need rows of whole float4s; the input-masked variant keeps one
    // crosspoint per lane (it loads twice the data per item and is not prefetched)
    typename std::conditional<VEC && !MIN, HaloVec<CP>, Halo<CP, MIN>>::type h;
    auto tile_at = [&](int tile, int& b, int& p0, int& q0) {
        b = tile / (th * tw);
        const int r = tile % (th * tw);
        p0 = (r / tw) * kTH;
        q0 = (r % tw) * kTW;
    };
    // without an input mask, the next tile's input is loaded while the current one is
    // computed; with one (twice the registers), each tile's input when it is staged
    constexpr bool PREFETCH = !MIN;
    if (PREFETCH && tr.first < tr.end) {
        int b, p0, q0;
        tile_at(tr.first, b, p0, q0);
        h.load(x + (int64_t)b * Cin * hw, nullptr, Cin, H, W, hw, p0, q0);
    }
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
        int b, p0, q0;
        tile_at(tile, b, p0, q0);
        if (!PREFETCH)
            h.load(x + (int64_t)b * Cin * hw, MIN ? mask_in + (int64_t)b * Cin * hw : nullptr, Cin, H, W, hw, p0, q0);
        // strip st of wave wv: tile row (4 wv + st) / kSR, columns from 16 ((4 wv + st) % kSR);
        // lane l holds crosspoints 4 (l / 16) .. + 3 of it.  The output mask is loaded
        // first, waited for while the input tile is staged, and kept as one bit per value
        // (bit 4 (NT st + nt) + v), so that no mask registers are live while the next
        // tile's input is in flight.
        fv4_t mk[4][NT];
        if (mask_out) {
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int sid = 4 * wv + st, p = p0 + sid / kSR, q = q0 + (sid % kSR) * 16 + 4 * g;
                    const int oc = nt * 16 + c16;
                    const bool ok = p < H && q < W && oc < Cout;
                    const int64_t o = ok ? ((int64_t)b * Cout + oc) * hw + (int64_t)p * W + q : 0;
                    if constexpr (vec) {
                        mk[st][nt] = *reinterpret_cast<const fv4_t*>(mask_out + o);
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v) mk[st][nt][v] = mask_out[ok && q + v < W ? o + v : 0];
                    }
                }
        }
        __syncthreads();                                  // the previous tile's reads are done
        h.store(xt, Cin, H, W, hw, p0, q0);
        __syncthreads();
        uint32_t mbits = 0;
        if (mask_out) {
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (mk[st][nt][v] > 0.0f) mbits |= 1u << (4 * (NT * st + nt) + v);
        }
        if (PREFETCH && tile + tr.step < tr.end) {
            int b1, p1, q1;
            tile_at(tile + tr.step, b1, p1, q1);
            h.load(x + (int64_t)b1 * Cin * hw, nullptr, Cin, H, W, hw, p1, q1);
        }
        fv4_t acc[4][NT];
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[st][nt] = fv4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < S; ++s) {
            // pairs beyond the last (j >= P) read a valid address and are zeroed after the read
            const int j = 4 * s + g, jj = j < P ? j : P - 1;
            const int t = jj / NCH, cc = jj % NCH;
            const int dy = t / 3, dx = t % 3;
            bf8_t wf[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                wf[nt] = *reinterpret_cast<const bf8_t*>(wl + (t * OC + nt * 16 + c16) * PS + 8 * cc);
                if (j >= P)
#pragma unroll
                    for (int i = 0; i < 8; ++i) wf[nt][i] = (__bf16)0.0f;
            }
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int sid = 4 * wv + st, pl = sid / kSR, ql = (sid % kSR) * 16;
                bf8_t a = *reinterpret_cast<const bf8_t*>(xt + ((pl + dy) * kHW + ql + c16 + dx) * PS + 8 * cc);
                if (j >= P)
#pragma unroll
                    for (int i = 0; i < 8; ++i) a[i] = (__bf16)0.0f;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[st][nt] = mma(a, wf[nt], acc[st][nt]);
            }
        }
        // D lane l item v: crosspoint 4 (l / 16) + v of the strip, output channel l % 16:
        // four consecutive crosspoints of one channel, one 16-byte store when W % 4 == 0
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int sid = 4 * wv + st, p = p0 + sid / kSR, q = q0 + (sid % kSR) * 16 + 4 * g;
            if (p >= H || q >= W) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int oc = nt * 16 + c16;
                if (oc >= Cout) continue;
                float* yo = y + ((int64_t)b * Cout + oc) * hw + (int64_t)p * W + q;
                fv4_t val = acc[st][nt];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (!BWD) {
                        val[v] += bo[nt];
                        if (relu) val[v] = fmaxf(val[v], 0.0f);
                    } else if (mask_out && !((mbits >> (4 * (NT * st + nt) + v)) & 1u)) {
                        val[v] = 0.0f;
                    }
                }
                if constexpr (vec) {
                    *reinterpret_cast<fv4_t*>(yo) = val;
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (q + v < W) yo[v] = val[v];
                }
            }
        }
    }
}

// Eight bfloat16 columns one to the left of M (the dword P before it supplies the first)
// and one to the right (the dword N after it supplies the last); two bfloat16 per dword,
// the lower column in the low half.
__device__ __forceinline__ bf8_t cols_left1(const bf8_t& M, uint32_t P)
{
    typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
    const u4_t a = __builtin_bit_cast(u4_t, M);
    const u4_t r{__builtin_amdgcn_alignbit(a[0], P, 16), __builtin_amdgcn_alignbit(a[1], a[0], 16),
                 __builtin_amdgcn_alignbit(a[2], a[1], 16), __builtin_amdgcn_alignbit(a[3], a[2], 16)};
    return __builtin_bit_cast(bf8_t, r);
}
__device__ __forceinline__ bf8_t cols_right1(const bf8_t& M, uint32_t N)
{
    typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
    const u4_t a = __builtin_bit_cast(u4_t, M);
    const u4_t r{__builtin_amdgcn_alignbit(a[1], a[0], 16), __builtin_amdgcn_alignbit(a[2], a[1], 16),
                 __builtin_amdgcn_alignbit(a[3], a[2], 16), __builtin_amdgcn_alignbit(N, a[3], 16)};
    return __builtin_bit_cast(bf8_t, r);
}

// Weight and bias gradient partial sums of one workgroup: NO, NC = tiles of 16 output
// and input channels (1 or 2 each).  part: [gridDim.x][O C 9 + O], laid out as the
// weights [o][c][tap], then the biases.  VEC: W % 4 == 0 and every array 16-byte
// aligned (16-byte loads).
template <int NO, int NC, bool VEC>
__global__ __launch_bounds__(256) void sg_wgrad_mfma_kernel(int B, int H, int W, int C, int O,
                                                            const float* __restrict__ x,
                                                            const float* __restrict__ gy,
                                                            const float* __restrict__ ymask,
                                                            float* __restrict__ part)
{
    // LDS, bfloat16: g (masked) as [16 NO channels][256 positions], row stride GS; the
    // input tile with its halo as [16 NC channels][10 rows][48 columns], halo column h
    // (input column q0 - 1 + h) at column h + 7, so that the 32 interior columns start
    // at an aligned column 8 (the other columns stay zero), channel stride CS.
    // GS = 132 words and CS = 244 words: the 16-byte reads of eight lanes (consecutive
    // channels) fall in distinct banks.
    constexpr int GS = kTH * kTW + 8;
    constexpr int RS = 48;
    constexpr int CS = kHH * RS + 8;
    constexpr int CR = 16 * NC;
    static_assert(kHW + 7 <= RS, "halo row fits");
    __shared__ __align__(16) __bf16 gs[16 * NO * GS];
    __shared__ __align__(16) __bf16 xs[CR * CS];
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, g = l >> 4, c16 = l & 15;
    const int mt = wv >> 1, nt = wv & 1;
    const bool active = mt < NO && nt < NC;
    // zeroed once: the padding columns and channels are never written again
    for (int e = threadIdx.x; e < CR * CS; e += 256) xs[e] = (__bf16)0.0f;
    fv4_t acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = fv4_t{0.0f, 0.0f, 0.0f, 0.0f};
    float accb = 0.0f;
    const int th = (H + kTH - 1) / kTH, tw = (W + kTW - 1) / kTW;
    const int tiles = B * th * tw;
    const int64_t hw = (int64_t)H * W;
    constexpr int GN = 16 * NO * kTH * kTW / 256;      // g elements per thread
    constexpr int XN = (CR * kHH * kHW + 255) / 256;   // input elements per thread
    constexpr int XB = 16;                              // input loads in flight per batch
    const TileRange tr = my_tiles(tiles);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
        const int b = tile / (th * tw), r = tile % (th * tw);
        const int p0 = (r / tw) * kTH, q0 = (r % tw) * kTW;
        __syncthreads();
        const float* gb = gy + (int64_t)b * O * hw;
        const float* mb = ymask ? ymask + (int64_t)b * O * hw : nullptr;
        const float* xb = x + (int64_t)b * C * hw;
        if constexpr (VEC) {
            // two passes, each with all its loads in flight: g, item (o, tile row, 4 columns),
            // one 16-byte load (and one of the mask); then the input
            typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
            constexpr int GI = 16 * NO * kTH * (kTW / 4) / 256;
            fv4_t gv[GI], gm[GI];
#pragma unroll
            for (int k = 0; k < GI; ++k) {
                const int e = k * 256 + threadIdx.x, o = e / (kTH * kTW / 4), rest = e % (kTH * kTW / 4);
                const int pp = p0 + rest / (kTW / 4), qq = q0 + 4 * (rest % (kTW / 4));
                const bool ok = o < O && pp < H && qq < W;
                const int64_t off = ok ? o * hw + (int64_t)pp * W + qq : 0;
                gv[k] = *reinterpret_cast<const fv4_t*>(gb + off);
                if (mb) gm[k] = *reinterpret_cast<const fv4_t*>(mb + off);
            }
#pragma unroll
            for (int k = 0; k < GI; ++k) {
                const int e = k * 256 + threadIdx.x, o = e / (kTH * kTW / 4), rest = e % (kTH * kTW / 4);
                const int pp = p0 + rest / (kTW / 4), qq = q0 + 4 * (rest % (kTW / 4));
                const bool ok = o < O && pp < H && qq < W;
                bf4_t t;
#pragma unroll
                for (int i = 0; i < 4; ++i) t[i] = (__bf16)((ok && (!mb || gm[k][i] > 0.0f)) ? gv[k][i] : 0.0f);
                *reinterpret_cast<bf4_t*>(gs + o * GS + 4 * rest) = t;
            }
            // input: interior item (c, halo row, 4 columns), one 16-byte load; edge item
            // (c, halo row, side), one load
            constexpr int XI = (CR * kHH * (kTW / 4) + 255) / 256;
            constexpr int XE = (CR * kHH * 2 + 255) / 256;
            fv4_t xv[XI];
            float xe[XE];
#pragma unroll
            for (int k = 0; k < XI; ++k) {
                const int e = k * 256 + threadIdx.x, c = e / (kHH * (kTW / 4)), rest = e % (kHH * (kTW / 4));
                const int pp = p0 + rest / (kTW / 4) - 1, qq = q0 + 4 * (rest % (kTW / 4));
                const bool ok = c < C && pp >= 0 && pp < H && qq < W;
                xv[k] = *reinterpret_cast<const fv4_t*>(xb + (ok ? c * hw + (int64_t)pp * W + qq : 0));
            }
#pragma unroll
            for (int k = 0; k < XE; ++k) {
                const int e = k * 256 + threadIdx.x, c = e / (2 * kHH), rr = (e >> 1) % kHH, side = e & 1;
                const int pp = p0 + rr - 1, qq = side ? q0 + kTW : q0 - 1;
                const bool ok = c < C && inside(pp, qq, H, W);
                xe[k] = xb[ok ? c * hw + (int64_t)pp * W + qq : 0];
            }
#pragma unroll
            for (int k = 0; k < XI; ++k) {
                const int e = k * 256 + threadIdx.x, c = e / (kHH * (kTW / 4)), rest = e % (kHH * (kTW / 4));
                if (c >= CR) continue;
                const int rr = rest / (kTW / 4), grp = rest % (kTW / 4);
                const int pp = p0 + rr - 1, qq = q0 + 4 * grp;
                const bool ok = c < C && pp >= 0 && pp < H && qq < W;
                bf4_t t;
#pragma unroll
                for (int i = 0; i < 4; ++i) t[i] = (__bf16)(ok ? xv[k][i] : 0.0f);
                *reinterpret_cast<bf4_t*>(xs + c * CS + rr * RS + 8 + 4 * grp) = t;
            }
#pragma unroll
            for (int k = 0; k < XE; ++k) {
                const int e = k * 256 + threadIdx.x, c = e / (2 * kHH), rr = (e >> 1) % kHH, side = e & 1;
                if (c >= CR) continue;
                const int pp = p0 + rr - 1, qq = side ? q0 + kTW : q0 - 1;
                const bool ok = c < C && inside(pp, qq, H, W);
                xs[c * CS + rr * RS + (side ? kHW + 6 : 7)] = (__bf16)(ok ? xe[k] : 0.0f);
            }
        } else {
            // g: element (o, position), positions fastest
            constexpr int GB = 16;                      // loads in flight per batch (32 with the mask)
#pragma unroll 1
            for (int k0 = 0; k0 < GN; k0 += GB) {
                float gv[GB], mk[GB];
                int64_t go[GB];
                bool gk[GB];
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    const int e = (k0 + k) * 256 + threadIdx.x, o = e >> 8, pos = e & 255;
                    const int pp = p0 + pos / kTW, qq = q0 + pos % kTW;
                    gk[k] = o < O && pp < H && qq < W;
                    go[k] = gk[k] ? o * hw + (int64_t)pp * W + qq : 0;
                    gv[k] = ld_or0(gb, go[k], gk[k]);
                }
                if (mb) {
#pragma unroll
                    for (int k = 0; k < GB; ++k) mk[k] = ld_or0(mb, go[k], gk[k]);
#pragma unroll
                    for (int k = 0; k < GB; ++k)
                        if (!(mk[k] > 0.0f)) gv[k] = 0.0f;
                }
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    const int e = (k0 + k) * 256 + threadIdx.x;
                    gs[(e >> 8) * GS + (e & 255)] = (__bf16)gv[k];
                }
            }
            // the input tile with its halo: element (c, halo row, halo column), columns fastest
#pragma unroll 1
            for (int k0 = 0; k0 < XN; k0 += XB) {
                float xv[XB];
#pragma unroll
                for (int k = 0; k < XB; ++k) {
                    const int e = (k0 + k) * 256 + threadIdx.x;
                    const int c = e / (kHH * kHW), rest = e % (kHH * kHW);
                    const int pp = p0 + rest / kHW - 1, qq = q0 + rest % kHW - 1;
                    const bool ok = k0 + k < XN && c < C && inside(pp, qq, H, W);
                    xv[k] = ld_or0(xb, ok ? c * hw + (int64_t)pp * W + qq : 0, ok);
                }
#pragma unroll
                for (int k = 0; k < XB; ++k) {
                    const int e = (k0 + k) * 256 + threadIdx.x;
                    const int c = e / (kHH * kHW), rest = e % (kHH * kHW);
                    if (k0 + k < XN && c < CR) xs[c * CS + (rest / kHW) * RS + rest % kHW + 7] = (__bf16)xv[k];
                }
            }
        }
        __syncthreads();
        if (active) {
            const int c = nt * 16 + c16;
#pragma unroll 2
            for (int s = 0; s < kTH * kTW / 32; ++s) {
                // A: g rows mt*16 + l%16, positions 32 s + 8 (l/16) .. + 7 (row p, columns q ..)
                const bf8_t a = *reinterpret_cast<const bf8_t*>(gs + (mt * 16 + c16) * GS + 32 * s + 8 * g);
                const int pos = 32 * s + 8 * g, p = pos / kTW, q = pos % kTW;
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    // B for taps (dy, 0..2): input row p + dy, halo columns q + dx .. q + dx + 7
                    // at LDS columns q + 7 + dx ..: the aligned eight at q + 8 (dx = 1) and
                    // the dwords before and after them
                    const __bf16* row = xs + c * CS + (p + dy) * RS + q;
                    const bf8_t xm = *reinterpret_cast<const bf8_t*>(row + 8);
                    const uint32_t xp = *reinterpret_cast<const uint32_t*>(row + 6);
                    const uint32_t xn = *reinterpret_cast<const uint32_t*>(row + 16);
                    acc[3 * dy] = mma(a, cols_left1(xm, xp), acc[3 * dy]);
                    acc[3 * dy + 1] = mma(a, xm, acc[3 * dy + 1]);
                    acc[3 * dy + 2] = mma(a, cols_right1(xm, xn), acc[3 * dy + 2]);
                }
            }
        }
        // bias: thread t sums 32 of the tile's positions of output channel t / 8
        {
            const int o = threadIdx.x >> 3, part = threadIdx.x & 7;
            if (o < 16 * NO) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bf8_t gv = *reinterpret_cast<const bf8_t*>(gs + o * GS + 32 * part + 8 * k);
#pragma unroll
                    for (int i = 0; i < 8; ++i) accb += (float)gv[i];
                }
            }
        }
    }
    // the eight partial bias sums of each channel, added in a fixed order
    accb += __shfl_xor(accb, 1, 8);
    accb += __shfl_xor(accb, 2, 8);
    accb += __shfl_xor(accb, 4, 8);
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
    if ((threadIdx.x & 7) == 0 && (threadIdx.x >> 3) < O) pw[ne + (threadIdx.x >> 3)] = accb;
}

template <bool BWD>
hipError_t launch_conv(int B, int H, int W, int Cin, int Cout, int relu, const float* x, const float* mask_in,
                       const float* w, const float* bias, const float* mask_out, float* y, hipStream_t s)
{
    const int64_t tiles = (int64_t)B * ((H + kTH - 1) / kTH) * ((W + kTW - 1) / kTW);
    // a multiple of 8 when there are at least 8 tiles (XCD-contiguous tile ranges)
    const int grid = (int)(tiles >= kConvGrid ? kConvGrid : tiles >= 8 ? tiles / 8 * 8 : tiles);
    const int cp = ((Cin + 7) / 8) * 8;
    const bool two = Cout > 16;
    auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const bool vec = (W & 3) == 0 && a16(x) && a16(mask_in) && a16(mask_out) && a16(y);
#define XB_CONV3(CPV, MINV, VECV)                                                                                 \
    if (two)                                                                                                       \
        hipLaunchKernelGGL((sg_conv_mfma_kernel<CPV, 2, BWD, MINV, VECV>), dim3(grid), dim3(256), 0, s, B, H, W,   \
                           Cin, Cout, relu, x, mask_in, w, bias, mask_out, y);                                      \
    else                                                                                                           \
        hipLaunchKernelGGL((sg_conv_mfma_kernel<CPV, 1, BWD, MINV, VECV>), dim3(grid), dim3(256), 0, s, B, H, W,   \
                           Cin, Cout, relu, x, mask_in, w, bias, mask_out, y);
#define XB_CONV2(CPV, MINV)                                                                                       \
    if (vec) {                                                                                                     \
        XB_CONV3(CPV, MINV, true)                                                                                  \
    } else {                                                                                                       \
        XB_CONV3(CPV, MINV, false)                                                                                 \
    }
#define XB_CONV(CPV)                                                                                               \
    if (BWD && mask_in) {                                                                                          \
        XB_CONV2(CPV, BWD)                                                                                         \
    } else {                                                                                                       \
        XB_CONV2(CPV, false)                                                                                       \
    }
    switch (cp) {
        case 8: XB_CONV(8) break;
        case 16: XB_CONV(16) break;
        case 24: XB_CONV(24) break;
        default: XB_CONV(32) break;
    }
#undef XB_CONV
#undef XB_CONV2
#undef XB_CONV3
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
    auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const bool vec = (W & 3) == 0 && a16(x) && a16(gy) && a16(ymask);
#define XB_WG(NOV, NCV)                                                                                            \
    if (vec)                                                                                                       \
        hipLaunchKernelGGL((sg_wgrad_mfma_kernel<NOV, NCV, true>), dim3(nparts), dim3(256), 0, s, B, H, W, C, O, x, \
                           gy, ymask, part);                                                                        \
    else                                                                                                           \
        hipLaunchKernelGGL((sg_wgrad_mfma_kernel<NOV, NCV, false>), dim3(nparts), dim3(256), 0, s, B, H, W, C, O,  \
                           x, gy, ymask, part);
    if (o2 && c2) {
        XB_WG(2, 2)
    } else if (o2) {
        XB_WG(2, 1)
    } else if (c2) {
        XB_WG(1, 2)
    } else {
        XB_WG(1, 1)
    }
#undef XB_WG
    return hipGetLastError();
}

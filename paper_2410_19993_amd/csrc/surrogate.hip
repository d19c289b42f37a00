// Learned current surrogate: features, 3x3 convolutions (forward, input
// gradient, weight gradient), column readout and loss, Adam, prediction.
//
// A small convolutional network over one crossbar's conductance map and inputs
// predicts the relative parasitic correction of each bit-line current,
// delta_j = (I_j - I0_j) / I0_j with I0 = G^T V, the currents without wire
// resistance (the zero-resistance limit of the nodal equations of Sec. II.A).
// The exact solver supplies the training targets and remains the reference.
//
// Layout: activations are float32 [B][C][H][W] (H = m rows, W = n columns);
// weights [O][C][3][3], biases [O].  All convolutions use zero padding of one
// crosspoint, so H and W are kept.  Every kernel handles any H, W >= 1 and
// C, O <= 32; a workgroup covers a 16 x 16 tile of crosspoints.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "xbar.h"

// bfloat16 matrix-core convolutions (surrogate_mfma.hip)
hipError_t xbk_sg_conv_forward_bf16(int B, int H, int W, int C, int O, int relu, const float* x, const float* w,
                                    const float* bias, float* y, hipStream_t s);
hipError_t xbk_sg_conv_backward_data_bf16(int B, int H, int W, int C, int O, const float* gy, const float* ymask,
                                          const float* w, const float* xmask, float* gx, hipStream_t s);
hipError_t xbk_sg_conv_backward_weight_bf16(int B, int H, int W, int C, int O, const float* x, const float* gy,
                                            const float* ymask, float* part, int nparts, hipStream_t s);

namespace {

constexpr int kMaxCh = XBAR_SG_MAX_CHANNELS;
constexpr int kMaxLine = XBAR_SG_MAX_LINE;
constexpr int kFeatures = XBAR_SG_FEATURES;
constexpr double kEstEps = XBAR_SG_EST_EPS;
constexpr double kEstMu = XBAR_SG_EST_MU;
constexpr double kEstSig = XBAR_SG_EST_SIGMA;
constexpr int kParts = 512;            // workgroups of the weight-gradient pass (partial sums; two fit a CU)
constexpr int kPer = (kMaxCh * kMaxCh * 9 + 255) / 256;

__device__ __forceinline__ bool in_grid(int p, int q, int H, int W) { return p >= 0 && p < H && q >= 0 && q < W; }

// X[b][0..6][i][j] = log10(G) + 5, 2 V_i, (r - 3) / 2, column and row position in
// [-1, 1], and the line totals 1e4 mean_j' G[i][j'] (row i) and 1e4 mean_i' G[i'][j] 2 V_i'
// (column j).  kFeatParts workgroups per sample (blockIdx.y), each writing a
// contiguous quarter of the rows; each forms all column totals and its rows'
// totals in LDS.
constexpr int kFeatParts = 4;

__global__ __launch_bounds__(256) void sg_features_kernel(int m, int n, const double* __restrict__ G,
                                                          const double* __restrict__ V, const double* __restrict__ r,
                                                          float* __restrict__ X)
{
    __shared__ double rows[kMaxLine], cols[kMaxLine];
    const int b = blockIdx.x;
    const int64_t mn = (int64_t)m * n;
    const double* gb = G + (int64_t)b * mn;
    const double* vb = V + (int64_t)b * m;
    const int per = (m + kFeatParts - 1) / kFeatParts;
    const int i0 = blockIdx.y * per, i1 = min(m, i0 + per);
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += gb[(int64_t)i * n + j];
        rows[i] = 1e4 * s / n;
    }
    for (int j = threadIdx.x; j < n; j += 256) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += gb[(int64_t)i * n + j] * 2.0 * vb[i];
        cols[j] = 1e4 * s / m;
    }
    __syncthreads();
    float* xb = X + (int64_t)b * kFeatures * mn;
    const float rr = (float)((r[b] - 3.0) * 0.5);
    for (int64_t e = (int64_t)i0 * n + threadIdx.x; e < (int64_t)i1 * n; e += 256) {
        const int i = (int)(e / n), j = (int)(e % n);
        xb[e] = (float)(log10(gb[e]) + 5.0);
        xb[mn + e] = (float)(2.0 * vb[i]);
        xb[2 * mn + e] = rr;
        xb[3 * mn + e] = n > 1 ? (float)(2.0 * j / (n - 1) - 1.0) : 0.0f;
        xb[4 * mn + e] = m > 1 ? (float)(2.0 * i / (m - 1) - 1.0) : 0.0f;
        xb[5 * mn + e] = (float)rows[i];
        xb[6 * mn + e] = (float)cols[j];
    }
}

// y[b][o] = bias[o] + sum_{c, dy, dx} w[o][c][dy][dx] x[b][c][p + dy - 1][q + dx - 1]  (ReLU optional).
// A workgroup covers 32 rows x 16 columns; each thread holds all O sums of two
// crosspoints 16 rows apart, so every weight read from LDS feeds two multiply-adds.
template <bool RELU>
__global__ __launch_bounds__(256) void sg_conv_fwd_kernel(int H, int W, int C, int O, const float* __restrict__ x,
                                                          const float* __restrict__ w,
                                                          const float* __restrict__ bias, float* __restrict__ y)
{
    __shared__ float ws[kMaxCh * kMaxCh * 9];
    __shared__ float bs[kMaxCh];
    for (int e = threadIdx.x; e < O * C * 9; e += 256) ws[e] = w[e];
    if (threadIdx.x < O) bs[threadIdx.x] = bias[threadIdx.x];
    __syncthreads();
    const int tw = (W + 15) / 16;
    const int p = (blockIdx.x / tw) * 32 + (threadIdx.x >> 4);
    const int q = (blockIdx.x % tw) * 16 + (threadIdx.x & 15);
    if (p >= H || q >= W) return;
    const bool two = p + 16 < H;
    const int64_t hw = (int64_t)H * W;
    const float* xb = x + (int64_t)blockIdx.y * C * hw;
    float acc[kMaxCh], acc2[kMaxCh];
#pragma unroll
    for (int o = 0; o < kMaxCh; ++o) acc[o] = acc2[o] = 0.0f;
    for (int c = 0; c < C; ++c) {
        const float* xc = xb + c * hw;
        float v[9], v2[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = p + t / 3 - 1, xx = q + t % 3 - 1;
            v[t] = in_grid(yy, xx, H, W) ? xc[(int64_t)yy * W + xx] : 0.0f;
            v2[t] = (two && in_grid(yy + 16, xx, H, W)) ? xc[(int64_t)(yy + 16) * W + xx] : 0.0f;
        }
        const float* wc = ws + c * 9;
#pragma unroll
        for (int o = 0; o < kMaxCh; ++o) {
            if (o < O) {
                float s = acc[o], s2 = acc2[o];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const float wv = wc[o * C * 9 + t];
                    s = fmaf(wv, v[t], s);
                    s2 = fmaf(wv, v2[t], s2);
                }
                acc[o] = s;
                acc2[o] = s2;
            }
        }
    }
    float* yb = y + (int64_t)blockIdx.y * O * hw + (int64_t)p * W + q;
#pragma unroll
    for (int o = 0; o < kMaxCh; ++o) {
        if (o < O) {
            float s = acc[o] + bs[o], s2 = acc2[o] + bs[o];
            if (RELU) {
                s = s > 0.0f ? s : 0.0f;
                s2 = s2 > 0.0f ? s2 : 0.0f;
            }
            yb[o * hw] = s;
            if (two) yb[o * hw + 16 * (int64_t)W] = s2;
        }
    }
}

// Gradient of the layer's output g = gy (times [ymask > 0] when the layer has a
// ReLU) with respect to its input:
//     gx[b][c][p][q] = sum_{o, dy, dx} w[o][c][dy][dx] g[b][o][p - dy + 1][q - dx + 1].
// As in the forward kernel, each thread takes two crosspoints 16 rows apart.  With
// xmask (the layer input, when it is a ReLU output) the result is written already
// multiplied by [xmask > 0], the gradient before the previous layer's ReLU, so the
// kernels that read it next need no mask.
__global__ __launch_bounds__(256) void sg_conv_bwd_data_kernel(int H, int W, int C, int O,
                                                               const float* __restrict__ gy,
                                                               const float* __restrict__ ymask,
                                                               const float* __restrict__ w,
                                                               const float* __restrict__ xmask,
                                                               float* __restrict__ gx)
{
    __shared__ float ws[kMaxCh * kMaxCh * 9];
    for (int e = threadIdx.x; e < O * C * 9; e += 256) ws[e] = w[e];
    __syncthreads();
    const int tw = (W + 15) / 16;
    const int p = (blockIdx.x / tw) * 32 + (threadIdx.x >> 4);
    const int q = (blockIdx.x % tw) * 16 + (threadIdx.x & 15);
    if (p >= H || q >= W) return;
    const bool two = p + 16 < H;
    const int64_t hw = (int64_t)H * W;
    const int64_t base = (int64_t)blockIdx.y * O * hw;
    float acc[kMaxCh], acc2[kMaxCh];
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c) acc[c] = acc2[c] = 0.0f;
    for (int o = 0; o < O; ++o) {
        const float* go = gy + base + o * hw;
        const float* mo = ymask ? ymask + base + o * hw : nullptr;
        float v[9], v2[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = p - t / 3 + 1, xx = q - t % 3 + 1;
            float g = 0.0f, g2 = 0.0f;
            if (in_grid(yy, xx, H, W)) {
                const int64_t off = (int64_t)yy * W + xx;
                g = go[off];
                if (mo && !(mo[off] > 0.0f)) g = 0.0f;
            }
            if (two && in_grid(yy + 16, xx, H, W)) {
                const int64_t off = (int64_t)(yy + 16) * W + xx;
                g2 = go[off];
                if (mo && !(mo[off] > 0.0f)) g2 = 0.0f;
            }
            v[t] = g;
            v2[t] = g2;
        }
        const float* wo = ws + o * C * 9;
#pragma unroll
        for (int c = 0; c < kMaxCh; ++c) {
            if (c < C) {
                float s = acc[c], s2 = acc2[c];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const float wv = wo[c * 9 + t];
                    s = fmaf(wv, v[t], s);
                    s2 = fmaf(wv, v2[t], s2);
                }
                acc[c] = s;
                acc2[c] = s2;
            }
        }
    }
    const int64_t xo = (int64_t)blockIdx.y * C * hw + (int64_t)p * W + q;
    float* gb = gx + xo;
    const float* xm = xmask ? xmask + xo : nullptr;
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c) {
        if (c < C) {
            float a = acc[c], a2 = acc2[c];
            if (xm) {
                if (!(xm[c * hw] > 0.0f)) a = 0.0f;
                if (two && !(xm[c * hw + 16 * (int64_t)W] > 0.0f)) a2 = 0.0f;
            }
            gb[c * hw] = a;
            if (two) gb[c * hw + 16 * (int64_t)W] = a2;
        }
    }
}

// Partial weight and bias gradients: workgroup k sums, over the 16 x 16 tiles
// k, k + kParts, ..., gw[o][c][dy][dx] = sum g[b][o][p][q] x[b][c][p + dy - 1][q + dx - 1]
// and gb[o] = sum g[b][o][p][q] into part[k][0 .. O C 9 + O).  The tile of g and
// the tile of x with its one-crosspoint halo are staged in LDS.  With G = 512 / C
// groups, thread t < G C owns input channel c = t % C and output channels
// o = t / C + G k (k < 2), all nine taps of each: it walks the tile row by row with
// the 3 x 3 window of x in registers, so each crosspoint costs three LDS reads of x
// and one of g per output channel for 9 multiply-adds per output channel.
constexpr int kXs = 18 * 18 + 1;        // LDS stride of a staged x channel (odd: spreads banks)
constexpr int kGs = 257;                // LDS stride of a staged g channel (odd: spreads banks)
constexpr int kWgT = 512;               // threads of a weight-gradient workgroup
constexpr int kOk = 2;                  // output channels per thread (512 / 32 = 16 groups of 2)

__global__ __launch_bounds__(kWgT) void sg_conv_bwd_weight_kernel(int B, int H, int W, int C, int O,
                                                                 const float* __restrict__ x,
                                                                 const float* __restrict__ gy,
                                                                 const float* __restrict__ ymask,
                                                                 float* __restrict__ part)
{
    __shared__ float gs[kMaxCh * kGs];          // [o][16 x 16]
    __shared__ float xs[kMaxCh * kXs];          // [c][18 x 18]
    const int ne = O * C * 9;
    const int tw = (W + 15) / 16, th = (H + 15) / 16;
    const int tiles = B * th * tw;
    const int64_t hw = (int64_t)H * W;
    const int groups = kWgT / C;
    const int c = threadIdx.x % C, og = threadIdx.x / C;
    const bool active = og < groups;
    int orow[kOk];
    float on[kOk];                              // 1 for an output channel this thread owns, else 0
#pragma unroll
    for (int k = 0; k < kOk; ++k) {
        const int o = og + groups * k;
        const bool own = active && o < O;
        on[k] = own ? 1.0f : 0.0f;
        orow[k] = (own ? o : 0) * kGs;          // a valid row of gs either way
    }
    float acc[kOk][9];
#pragma unroll
    for (int k = 0; k < kOk; ++k)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[k][t] = 0.0f;
    float accb = 0.0f;
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int b = t / (th * tw), r = t % (th * tw);
        const int p0 = (r / tw) * 16, q0 = (r % tw) * 16;
        __syncthreads();                        // the previous tile's LDS reads are done
        for (int e = threadIdx.x; e < O * 256; e += kWgT) {
            const int o = e >> 8, p = p0 + ((e & 255) >> 4), q = q0 + (e & 15);
            float g = 0.0f;
            if (p < H && q < W) {
                const int64_t off = ((int64_t)b * O + o) * hw + (int64_t)p * W + q;
                g = gy[off];
                if (ymask && !(ymask[off] > 0.0f)) g = 0.0f;
            }
            gs[o * kGs + (e & 255)] = g;
        }
        for (int e = threadIdx.x; e < C * 324; e += kWgT) {
            const int cc = e / 324, k = e % 324;
            const int p = p0 + k / 18 - 1, q = q0 + k % 18 - 1;
            xs[cc * kXs + k] = in_grid(p, q, H, W) ? x[((int64_t)b * C + cc) * hw + (int64_t)p * W + q] : 0.0f;
        }
        __syncthreads();
        if (active) {
            const float* xc = xs + c * kXs;
            for (int pr = 0; pr < 16; ++pr) {
                const float* xr = xc + pr * 18;
                float a0 = xr[0], a1 = xr[18], a2 = xr[36];
                float b0 = xr[1], b1 = xr[19], b2 = xr[37];
#pragma unroll
                for (int pc = 0; pc < 16; ++pc) {
                    const float c0 = xr[pc + 2], c1 = xr[pc + 20], c2 = xr[pc + 38];
#pragma unroll
                    for (int k = 0; k < kOk; ++k) {
                        const float g = on[k] * gs[orow[k] + pr * 16 + pc];
                        acc[k][0] = fmaf(g, a0, acc[k][0]);
                        acc[k][1] = fmaf(g, b0, acc[k][1]);
                        acc[k][2] = fmaf(g, c0, acc[k][2]);
                        acc[k][3] = fmaf(g, a1, acc[k][3]);
                        acc[k][4] = fmaf(g, b1, acc[k][4]);
                        acc[k][5] = fmaf(g, c1, acc[k][5]);
                        acc[k][6] = fmaf(g, a2, acc[k][6]);
                        acc[k][7] = fmaf(g, b2, acc[k][7]);
                        acc[k][8] = fmaf(g, c2, acc[k][8]);
                    }
                    a0 = b0; b0 = c0;
                    a1 = b1; b1 = c1;
                    a2 = b2; b2 = c2;
                }
            }
        }
        if (threadIdx.x < O) {
            float sb = 0.0f;
            for (int e = 0; e < 256; ++e) sb += gs[threadIdx.x * kGs + e];
            accb += sb;
        }
    }
    float* pw = part + (int64_t)blockIdx.x * (ne + O);
#pragma unroll
    for (int k = 0; k < kOk; ++k) {
        const int o = og + groups * k;
        if (active && o < O)
#pragma unroll
            for (int t = 0; t < 9; ++t) pw[(o * C + c) * 9 + t] = acc[k][t];
    }
    if (threadIdx.x < O) pw[ne + threadIdx.x] = accb;
}

// gw[e] = sum over the partials; e >= ne: gb.  Each workgroup takes 16 entries; lane
// l of an entry adds the partials l, l + 16, ... in order, and the sixteen sums are
// then added in lane order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void sg_reduce_parts_kernel(int nparts, int ne, int O,
                                                              const float* __restrict__ part,
                                                              float* __restrict__ gw, float* __restrict__ gb)
{
    __shared__ float red[16][16];
    const int le = threadIdx.x & 15, lp = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + le;
    float s = 0.0f;
    if (e < ne + O) {
        // eight partials in flight at a time, added in the same order as one at a time
        const int64_t stride = ne + O;
        int k = lp;
        for (; k + 7 * 16 < nparts; k += 8 * 16) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = part[(int64_t)(k + 16 * i) * stride + e];
#pragma unroll
            for (int i = 0; i < 8; ++i) s += v[i];
        }
        for (; k < nparts; k += 16) s += part[(int64_t)k * stride + e];
    }
    red[lp][le] = s;
    __syncthreads();
    if (lp == 0 && e < ne + O) {
        float t = red[0][le];
        for (int k = 1; k < 16; ++k) t += red[k][le];
        if (e < ne) gw[e] = t;
        else gb[e - ne] = t;
    }
}

// Column readouts of the last map Y[b][0..1] and the loss gradient:
// yhat_j = mean_i Y[b][0][i][j], s_j = mean_i Y[b][1][i][j], e_j = yhat_j - delta_j,
// t_j = (log(e_j^2 + eps) - mu) / sigma (held constant);  gY[b][0][i][j] = 2 e_j / (B n m),
// gY[b][1][i][j] = lam 2 (s_j - t_j) / (B n m);  err2[b] = {sum_j e_j^2, sum_j (s_j - t_j)^2}.
// One workgroup per sample.
__global__ __launch_bounds__(256) void sg_readout_loss_kernel(int B, int m, int n, const float* __restrict__ Y,
                                                              const double* __restrict__ delta, double lam,
                                                              float* __restrict__ gY, double* __restrict__ err2)
{
    __shared__ double red[2][256];
    const int b = blockIdx.x;
    const int64_t mn = (int64_t)m * n;
    const float* y0 = Y + (int64_t)b * 2 * mn;
    const float* y1 = y0 + mn;
    float* g0 = gY + (int64_t)b * 2 * mn;
    float* g1 = g0 + mn;
    const double scale = 2.0 / ((double)B * n * m);
    double e2 = 0.0, d2 = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i < m; ++i) {
            s0 += y0[(int64_t)i * n + j];
            s1 += y1[(int64_t)i * n + j];
        }
        const double e = s0 / m - delta[(int64_t)b * n + j];
        const double d = s1 / m - (log(e * e + kEstEps) - kEstMu) / kEstSig;
        e2 += e * e;
        d2 += d * d;
        const float ga = (float)(scale * e), gb = (float)(lam * scale * d);
        for (int i = 0; i < m; ++i) {
            g0[(int64_t)i * n + j] = ga;
            g1[(int64_t)i * n + j] = gb;
        }
    }
    red[0][threadIdx.x] = e2;
    red[1][threadIdx.x] = d2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        err2[2 * b] = red[0][0];
        err2[2 * b + 1] = red[1][0];
    }
}

// Adam with bias correction; c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void sg_adam_kernel(int64_t count, float* __restrict__ p, const float* __restrict__ g,
                               float* __restrict__ m1, float* __restrict__ m2, float lr, float b1, float b2,
                               float eps, float c1, float c2)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float ge = g[e];
    const float a = b1 * m1[e] + (1.0f - b1) * ge;
    const float v = b2 * m2[e] + (1.0f - b2) * ge * ge;
    m1[e] = a;
    m2[e] = v;
    p[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Training targets: delta[e] = (I[e] - I0[e]) / I0[e] over B n entries.
__global__ void sg_targets_kernel(int64_t count, const double* __restrict__ I, const double* __restrict__ I0,
                                  double* __restrict__ delta)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        delta[e] = (I[e] - I0[e]) / I0[e];
}

// Fixed-order maximum over a workgroup of 256 (NaN above everything).
// Maximum that keeps NaN (fmax drops a NaN as soon as a number follows it).
__device__ inline double nan_max(double a, double b)
{
    return (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
}

__device__ double wg_max(double v, double* red)
{
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return nan_max(nan_max(red[0], red[1]), nan_max(red[2], red[3]));
}

// Calibration ratio of sample b (one workgroup): the largest relative current error of
// the prediction Ip over the columns with a nonzero exact current I, divided by the
// largest error estimate; NaN when no column has I != 0, when either maximum is not
// finite, or when the estimate's maximum is not positive (such samples do not enter
// the quantile).
__global__ __launch_bounds__(256) void sg_calib_ratio_kernel(int n, const double* __restrict__ Ip,
                                                             const double* __restrict__ I,
                                                             const double* __restrict__ est,
                                                             double* __restrict__ ratio)
{
    __shared__ double red[4];
    const int64_t o = (int64_t)blockIdx.x * n;
    double worst = 0.0, emax = 0.0, live = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const double x = I[o + j];
        if (x != 0.0) {
            const double r = fabs(Ip[o + j] - x) / fabs(x);
            worst = nan_max(worst, r);
            live = 1.0;
        }
        emax = nan_max(emax, est[o + j]);
    }
    worst = wg_max(worst, red);
    emax = wg_max(emax, red);
    live = wg_max(live, red);
    if (threadIdx.x == 0) {
        const bool ok = live > 0.0 && isfinite(worst) && isfinite(emax) && emax > 0.0;
        ratio[blockIdx.x] = ok ? worst / emax : __builtin_nan("");
    }
}

// Routing of checked predictions (one workgroup per sample): flag[b] = 1 (solve it
// exactly) unless kappa times the largest error estimate is a number <= tol, every
// predicted current is finite, every conductance is finite and positive and every
// input is finite.
__global__ __launch_bounds__(256) void sg_route_kernel(int m, int n, const double* __restrict__ G,
                                                       const double* __restrict__ V, const double* __restrict__ I,
                                                       const double* __restrict__ est, double kappa, double tol,
                                                       int* __restrict__ flag)
{
    __shared__ double red[4];
    const int b = blockIdx.x;
    double bad = 0.0, emax = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        emax = nan_max(emax, est[(int64_t)b * n + j]);
        if (!isfinite(I[(int64_t)b * n + j])) bad = 1.0;
    }
    const int64_t mn = (int64_t)m * n;
    for (int64_t k = threadIdx.x; k < mn; k += 256) {
        const double g = G[(int64_t)b * mn + k];
        if (!(isfinite(g) && g > 0.0)) bad = 1.0;
    }
    for (int i = threadIdx.x; i < m; i += 256)
        if (!isfinite(V[(int64_t)b * m + i])) bad = 1.0;
    bad = wg_max(bad, red);
    emax = wg_max(emax, red);
    if (threadIdx.x == 0) flag[b] = (bad > 0.0 || !(kappa * emax <= tol)) ? 1 : 0;
}

// I[b][j] = (sum_i G[b][i][j] V[b][i]) (1 + yhat_j), yhat_j = mean_i Y[b][0][i][j];
// est[b][j] = exp((sigma mean_i Y[b][1][i][j] + mu) / 2) / |1 + yhat_j|, the predicted
// relative current error (skipped when est is null).
__global__ void sg_predict_kernel(int B, int m, int n, const float* __restrict__ Y, const double* __restrict__ G,
                                  const double* __restrict__ V, double* __restrict__ I, double* __restrict__ est)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (j >= n) return;
    const int64_t mn = (int64_t)m * n;
    const double* gb = G + (int64_t)b * mn;
    const float* y0 = Y + (int64_t)b * 2 * mn;
    const float* y1 = y0 + mn;
    const double* vb = V + (int64_t)b * m;
    double i0 = 0.0, s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < m; ++i) {
        i0 += gb[(int64_t)i * n + j] * vb[i];
        s0 += y0[(int64_t)i * n + j];
        s1 += y1[(int64_t)i * n + j];
    }
    I[(int64_t)b * n + j] = i0 * (1.0 + s0 / m);
    if (est) est[(int64_t)b * n + j] = exp(0.5 * (kEstSig * s1 / m + kEstMu)) / fabs(1.0 + s0 / m);
}

bool shape_ok(int32_t B, int32_t H, int32_t W) { return B >= 1 && B <= 65535 && H >= 1 && W >= 1; }
bool ch_ok(int32_t C, int32_t O) { return C >= 1 && C <= kMaxCh && O >= 1 && O <= kMaxCh; }

// [a, a + na) and [b, b + nb) share a byte
bool overlap(const void* a, int64_t na, const void* b, int64_t nb)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + (uintptr_t)nb && y < x + (uintptr_t)na;
}

xbar_status launched()
{
    if (hipGetLastError() != hipSuccess) return XBAR_ERR_DEVICE;
    return XBAR_OK;
}

dim3 tile_grid(int B, int H, int W) { return dim3(((H + 15) / 16) * ((W + 15) / 16), B); }
dim3 tall_grid(int B, int H, int W) { return dim3(((H + 31) / 32) * ((W + 15) / 16), B); }

}  // namespace

namespace {

// The weight gradient's two launches: per-workgroup partial sums into `work`, then
// their fixed-order reduction into gw and gb.
xbar_status bwd_weight_launch(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* x,
                              const float* gy, const float* ymask, float* gw, float* gb, float* work, int nparts,
                              hipStream_t s)
{
    const int ne = O * C * 9;
    hipLaunchKernelGGL(sg_conv_bwd_weight_kernel, dim3(nparts), dim3(kWgT), 0, s, B, H, W, C, O, x, gy, ymask, work);
    if (hipGetLastError() != hipSuccess) return XBAR_ERR_DEVICE;
    hipLaunchKernelGGL(sg_reduce_parts_kernel, dim3((ne + O + 15) / 16), dim3(256), 0, s, nparts, ne, O, work, gw,
                       gb);
    return launched();
}

int bwd_weight_parts(int32_t B, int32_t H, int32_t W)
{
    const int64_t tiles = (int64_t)B * ((H + 15) / 16) * ((W + 15) / 16);
    return (int)(tiles < kParts ? tiles : kParts);
}

// Workspace of the allocation-free weight gradient: the partial sums for the largest
// channel counts, a file-scope device array.  Each GPU the library runs on holds its
// own copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in), looked up once per device.
constexpr int64_t kSgScratchFloats = (int64_t)kParts * (XBAR_SG_MAX_CHANNELS * XBAR_SG_MAX_CHANNELS * 9 +
                                                         XBAR_SG_MAX_CHANNELS);
}  // namespace

static __device__ __align__(256) float scratch[kSgScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
float* scratch_at[kMaxDevices] = {};

float* scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_at[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_at[dev] = static_cast<float*>(p);
    }
    return scratch_at[dev];
}

}  // namespace

extern "C" {

int64_t xbar_sg_workspace_floats(int32_t C, int32_t O)
{
    if (!ch_ok(C, O)) return -1;
    return (int64_t)kParts * (O * C * 9 + O);
}

xbar_status xbar_sg_features(int32_t B, int32_t m, int32_t n, const double* G, const double* V, const double* r,
                             float* X, void* hip_stream)
{
    if (!shape_ok(B, m, n) || m > kMaxLine || n > kMaxLine || !G || !V || !r || !X) return XBAR_ERR_ARG;
    const int64_t total = (int64_t)B * m * n, nx = total * kFeatures * 4;
    if (overlap(X, nx, G, total * 8) || overlap(X, nx, V, (int64_t)B * m * 8) || overlap(X, nx, r, (int64_t)B * 8))
        return XBAR_ERR_ARG;
    hipLaunchKernelGGL(sg_features_kernel, dim3(B, kFeatParts), dim3(256), 0, reinterpret_cast<hipStream_t>(hip_stream),
                       m, n, G, V, r, X);
    return launched();
}

xbar_status xbar_sg_conv_forward(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, int32_t relu, const float* x,
                                 const float* w, const float* bias, float* y, void* hip_stream)
{
    if (!shape_ok(B, H, W) || !ch_ok(C, O) || !x || !w || !bias || !y) return XBAR_ERR_ARG;
    const int64_t hw = (int64_t)H * W;
    if (overlap(y, (int64_t)B * O * hw * 4, x, (int64_t)B * C * hw * 4) ||
        overlap(y, (int64_t)B * O * hw * 4, w, (int64_t)O * C * 36) || overlap(y, (int64_t)B * O * hw * 4, bias, O * 4))
        return XBAR_ERR_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (relu)
        hipLaunchKernelGGL(sg_conv_fwd_kernel<true>, tall_grid(B, H, W), dim3(256), 0, s, H, W, C, O, x, w, bias, y);
    else
        hipLaunchKernelGGL(sg_conv_fwd_kernel<false>, tall_grid(B, H, W), dim3(256), 0, s, H, W, C, O, x, w, bias, y);
    return launched();
}

xbar_status xbar_sg_conv_backward_data(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* gy,
                                       const float* ymask, const float* w, const float* xmask, float* gx,
                                       void* hip_stream)
{
    if (!shape_ok(B, H, W) || !ch_ok(C, O) || !gy || !w || !gx) return XBAR_ERR_ARG;
    const int64_t hw = (int64_t)H * W, nx = (int64_t)B * C * hw * 4, ny = (int64_t)B * O * hw * 4;
    if (overlap(gx, nx, gy, ny) || (ymask && overlap(gx, nx, ymask, ny)) || overlap(gx, nx, w, (int64_t)O * C * 36) ||
        (xmask && overlap(gx, nx, xmask, nx)))
        return XBAR_ERR_ARG;
    hipLaunchKernelGGL(sg_conv_bwd_data_kernel, tall_grid(B, H, W), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), H, W, C, O, gy, ymask, w, xmask, gx);
    return launched();
}


xbar_status xbar_sg_conv_forward_bf16(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, int32_t relu,
                                      const float* x, const float* w, const float* bias, float* y, void* hip_stream)
{
    if (!shape_ok(B, H, W) || !ch_ok(C, O) || !x || !w || !bias || !y) return XBAR_ERR_ARG;
    const int64_t hw = (int64_t)H * W;
    if (overlap(y, (int64_t)B * O * hw * 4, x, (int64_t)B * C * hw * 4) ||
        overlap(y, (int64_t)B * O * hw * 4, w, (int64_t)O * C * 36) || overlap(y, (int64_t)B * O * hw * 4, bias, O * 4))
        return XBAR_ERR_ARG;
    if (xbk_sg_conv_forward_bf16(B, H, W, C, O, relu, x, w, bias, y, reinterpret_cast<hipStream_t>(hip_stream)) !=
        hipSuccess)
        return XBAR_ERR_DEVICE;
    return launched();
}

xbar_status xbar_sg_conv_backward_data_bf16(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* gy,
                                            const float* ymask, const float* w, const float* xmask, float* gx,
                                            void* hip_stream)
{
    if (!shape_ok(B, H, W) || !ch_ok(C, O) || !gy || !w || !gx) return XBAR_ERR_ARG;
    const int64_t hw = (int64_t)H * W, nx = (int64_t)B * C * hw * 4, ny = (int64_t)B * O * hw * 4;
    if (overlap(gx, nx, gy, ny) || (ymask && overlap(gx, nx, ymask, ny)) || overlap(gx, nx, w, (int64_t)O * C * 36) ||
        (xmask && overlap(gx, nx, xmask, nx)))
        return XBAR_ERR_ARG;
    if (xbk_sg_conv_backward_data_bf16(B, H, W, C, O, gy, ymask, w, xmask, gx,
                                       reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return XBAR_ERR_DEVICE;
    return launched();
}

xbar_status xbar_sg_conv_backward_weight_bf16(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* x,
                                              const float* gy, const float* ymask, float* gw, float* gb, float* work,
                                              int64_t work_floats, void* hip_stream)
{
    if (!shape_ok(B, H, W) || !ch_ok(C, O) || !x || !gy || !gw || !gb || !work) return XBAR_ERR_ARG;
    const int ne = O * C * 9;
    const int nparts = bwd_weight_parts(B, H, W);
    if (work_floats < (int64_t)nparts * (ne + O)) return XBAR_ERR_ARG;
    const int64_t nw = (int64_t)nparts * (ne + O) * 4;
    if (overlap(work, nw, gw, ne * 4) || overlap(work, nw, gb, O * 4) || overlap(gw, ne * 4, gb, O * 4))
        return XBAR_ERR_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (xbk_sg_conv_backward_weight_bf16(B, H, W, C, O, x, gy, ymask, work, nparts, s) != hipSuccess)
        return XBAR_ERR_DEVICE;
    hipLaunchKernelGGL(sg_reduce_parts_kernel, dim3((ne + O + 15) / 16), dim3(256), 0, s, nparts, ne, O, work, gw,
                       gb);
    return launched();
}

xbar_status xbar_sg_conv_backward_weight(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* x,
                                         const float* gy, const float* ymask, float* gw, float* gb, float* work,
                                         int64_t work_floats, void* hip_stream)
{
    if (!shape_ok(B, H, W) || !ch_ok(C, O) || !x || !gy || !gw || !gb || !work) return XBAR_ERR_ARG;
    const int ne = O * C * 9;
    const int nparts = bwd_weight_parts(B, H, W);
    if (work_floats < (int64_t)nparts * (ne + O)) return XBAR_ERR_ARG;
    const int64_t nw = (int64_t)nparts * (ne + O) * 4;
    if (overlap(work, nw, gw, ne * 4) || overlap(work, nw, gb, O * 4) || overlap(gw, ne * 4, gb, O * 4))
        return XBAR_ERR_ARG;
    return bwd_weight_launch(B, H, W, C, O, x, gy, ymask, gw, gb, work, nparts,
                             reinterpret_cast<hipStream_t>(hip_stream));
}

xbar_status xbar_sg_conv_backward_weight_noalloc(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O,
                                                 const float* x, const float* gy, const float* ymask, float* gw,
                                                 float* gb, void* hip_stream)
{
    if (!shape_ok(B, H, W) || !ch_ok(C, O) || !x || !gy || !gw || !gb) return XBAR_ERR_ARG;
    const int ne = O * C * 9;
    const int nparts = bwd_weight_parts(B, H, W);
    if ((int64_t)nparts * (ne + O) > kSgScratchFloats) return XBAR_ERR_ARG;
    if (overlap(gw, ne * 4, gb, O * 4)) return XBAR_ERR_ARG;
    float* ws = scratch_ptr();
    if (ws == nullptr) return XBAR_ERR_DEVICE;
    return bwd_weight_launch(B, H, W, C, O, x, gy, ymask, gw, gb, ws, nparts,
                             reinterpret_cast<hipStream_t>(hip_stream));
}

xbar_status xbar_sg_readout_loss(int32_t B, int32_t m, int32_t n, const float* Y, const double* delta, double lam,
                                 float* gY, double* err2, void* hip_stream)
{
    if (!shape_ok(B, m, n) || !Y || !delta || !gY || !err2 || !(lam >= 0.0)) return XBAR_ERR_ARG;
    const int64_t ny = (int64_t)B * 2 * m * n * 4;
    if (overlap(gY, ny, Y, ny) || overlap(gY, ny, delta, (int64_t)B * n * 8) ||
        overlap(err2, (int64_t)B * 16, gY, ny) || overlap(err2, (int64_t)B * 16, Y, ny))
        return XBAR_ERR_ARG;
    hipLaunchKernelGGL(sg_readout_loss_kernel, dim3(B), dim3(256), 0, reinterpret_cast<hipStream_t>(hip_stream), B, m,
                       n, Y, delta, lam, gY, err2);
    return launched();
}

xbar_status xbar_sg_adam(int64_t count, float* p, const float* g, float* m1, float* m2, double lr, double b1,
                         double b2, double eps, int32_t t, void* hip_stream)
{
    if (count < 1 || !p || !g || !m1 || !m2 || t < 1 || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) ||
        !(eps > 0))
        return XBAR_ERR_ARG;
    const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
    hipLaunchKernelGGL(sg_adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), count, p, g, m1, m2, (float)lr, (float)b1,
                       (float)b2, (float)eps, (float)c1, (float)c2);
    return launched();
}

xbar_status xbar_sg_predict(int32_t B, int32_t m, int32_t n, const float* Y, const double* G, const double* V,
                            double* I, double* est, void* hip_stream)
{
    if (!shape_ok(B, m, n) || !Y || !G || !V || !I) return XBAR_ERR_ARG;
    const int64_t ni = (int64_t)B * n * 8;
    if (overlap(I, ni, Y, (int64_t)B * 2 * m * n * 4) || overlap(I, ni, G, (int64_t)B * m * n * 8) ||
        overlap(I, ni, V, (int64_t)B * m * 8) || (est && overlap(est, ni, I, ni)) ||
        (est && overlap(est, ni, Y, (int64_t)B * 2 * m * n * 4)))
        return XBAR_ERR_ARG;
    hipLaunchKernelGGL(sg_predict_kernel, dim3((n + 255) / 256, B), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), B, m, n, Y, G, V, I, est);
    return launched();
}

xbar_status xbar_sg_targets(int32_t S, int32_t n, const double* I, const double* I0, double* delta,
                            void* hip_stream)
{
    if (S < 1 || n < 1 || !I || !I0 || !delta) return XBAR_ERR_ARG;
    const int64_t nb = (int64_t)S * n * 8;
    if (overlap(delta, nb, I, nb) || overlap(delta, nb, I0, nb)) return XBAR_ERR_ARG;
    const int64_t count = (int64_t)S * n;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(sg_targets_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(hip_stream), count, I, I0, delta);
    return launched();
}

xbar_status xbar_sg_calib_ratios(int32_t B, int32_t n, const double* Ip, const double* I, const double* est,
                                 double* ratio, void* hip_stream)
{
    if (B < 1 || B > 65535 || n < 1 || !Ip || !I || !est || !ratio) return XBAR_ERR_ARG;
    const int64_t nb = (int64_t)B * n * 8;
    if (overlap(ratio, (int64_t)B * 8, Ip, nb) || overlap(ratio, (int64_t)B * 8, I, nb) ||
        overlap(ratio, (int64_t)B * 8, est, nb))
        return XBAR_ERR_ARG;
    hipLaunchKernelGGL(sg_calib_ratio_kernel, dim3(B), dim3(256), 0, reinterpret_cast<hipStream_t>(hip_stream), n,
                       Ip, I, est, ratio);
    return launched();
}

xbar_status xbar_sg_route(int32_t B, int32_t m, int32_t n, const double* G, const double* V, const double* I,
                          const double* est, double kappa, double tol, int32_t* flag, void* hip_stream)
{
    if (!shape_ok(B, m, n) || !G || !V || !I || !est || !flag) return XBAR_ERR_ARG;
    if (!(kappa >= 0.0) || !(tol >= 0.0)) return XBAR_ERR_ARG;
    hipLaunchKernelGGL(sg_route_kernel, dim3(B), dim3(256), 0, reinterpret_cast<hipStream_t>(hip_stream), m, n, G, V,
                       I, est, kappa, tol, flag);
    return launched();
}

}  // extern "C"

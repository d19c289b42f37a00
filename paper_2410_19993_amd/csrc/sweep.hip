// Forward and back substitution over the row blocks (Sec. II.C: L y = I then
// U v = y, for every input vector of a batch, Sec. III.A/III.D), in the
// twisted order of the factorization (top chain rows 0..kt-1, bottom chain
// rows m-1..kt+1, twist row kt = m/2), with H_i the stored pivot inverses:
//   forward, top:    y_0 = f_0,        z_i = H_i y_i,  y_{i+1} = f_{i+1} + g_bl z_i
//   forward, bottom: y_{m-1} = f_{m-1}, z_i = H_i y_i,  y_{i-1} = f_{i-1} + g_bl z_i
//   twist:           u_kt = H_kt (f_kt + g_bl z_{kt-1} + g_bl z_{kt+1})
//   back, up:        u_i = z_i + g_bl H_i u_{i+1}   (i = kt-1 .. 0)
//   back, down:      u_i = z_i + g_bl H_i u_{i-1}   (i = kt+1 .. m-1)
// with f_i = V_i c_i.  Output currents are I_j = g_sense u_{m-1, j}, and the
// word-line voltages of row i follow from its tridiagonal block,
//   T_i w_i = g_src V_i e_0 + Gam_i u_i.
//
// Input vectors are independent, so each workgroup owns a slab of 16 of
// them for the whole sweep: no grid synchronisation at all.  Per row block
// it computes an (n_p x n_p) x (n_p x 16) product on the matrix cores: H_i
// streams from L2/HBM straight into registers as MFMA A fragments, and the
// 16-column right-hand-side panel sits in LDS (H_i fragment-tiled, so each
// load instruction of a wave reads 1 KB of contiguous memory).  W waves (8 when n_p/64 is
// even, else 4) each own a band of TW = 4 n_p / (64 W) tiles of 16 rows, so
// that the accumulators and one chunk of prefetched H stay in registers.
#include "common.h"

namespace xbk {

template <typename T> struct Vec4;
template <> struct Vec4<double> { using type = d4_t; };
template <> struct Vec4<float> { using type = f4_t; };

// k position inside a CPR row (16-chunk permuted)
template <typename T>
__device__ __host__ inline int pos(int k) { return (k & ~15) + Frag<T>::slot(k & 15); }

// A-operand fragment of FRG tile (tr, tk) of an n_p x n_p block (kt = n_p / 16):
// one contiguous 1 KB region per 16-byte load instruction.
template <typename T>
__device__ __forceinline__ typename Vec4<T>::type load_frag(const T* __restrict__ M, int kt, int tr, int tk, int l)
{
    using v4 = typename Vec4<T>::type;
    const T* p = M + ((int64_t)tr * kt + tk) * 256;
    if constexpr (sizeof(T) == 8) {
        typedef double d2_t __attribute__((ext_vector_type(2)));
        const d2_t lo = *reinterpret_cast<const d2_t*>(p + 2 * l);
        const d2_t hi = *reinterpret_cast<const d2_t*>(p + 128 + 2 * l);
        return v4{lo[0], lo[1], hi[0], hi[1]};
    } else {
        return *reinterpret_cast<const v4*>(p + 4 * l);
    }
}

// acc[t] = (rows of tile t of this wave) x panel, K = n_p in chunks of 16;
// H_i is FRG, the panel is [column][CPR position].
template <typename T, int NT, int TW>
__device__ __forceinline__ void panel_product(typename Frag<T>::acc_t (&acc)[TW], const T* __restrict__ Hi,
                                              const T* ybuf, int ldy, int w, int l)
{
    using v4 = typename Vec4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    constexpr int n_p = 64 * NT;
    constexpr int KC = n_p / 16;             // even
    // float fragments are half the size: keep two chunks of H in flight instead of one
    constexpr int D = sizeof(T) == 4 ? 2 : 1;
    const int q = l >> 4, r = l & 15;
#pragma unroll
    for (int t = 0; t < TW; ++t) acc[t] = acc_t{0, 0, 0, 0};
    v4 cur[D][TW], nxt[D][TW];
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int t = 0; t < TW; ++t) cur[d][t] = load_frag<T>(Hi, KC, TW * w + t, d, l);
    for (int K = 0; K < KC; K += D) {
        const bool more = K + D < KC;
        if (more) {
#pragma unroll
            for (int d = 0; d < D; ++d)
#pragma unroll
                for (int t = 0; t < TW; ++t) nxt[d][t] = load_frag<T>(Hi, KC, TW * w + t, K + D + d, l);
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const v4 bv = *reinterpret_cast<const v4*>(ybuf + r * ldy + 16 * (K + d) + 4 * q);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < TW; ++t) acc[t] = Frag<T>::mma(cur[d][t][s], bv[s], acc[t]);
        }
        if (more) {
#pragma unroll
            for (int d = 0; d < D; ++d)
#pragma unroll
                for (int t = 0; t < TW; ++t) cur[d][t] = nxt[d][t];
        }
    }
}

// ---------------------------------------------------------------------------
// Tridiagonal solves T_i w = d split over LANES lanes per vector.
// Lane s owns the contiguous segment [s << lg, (s+1) << lg); element j lives at
// LDS index j + (j >> lg) (one pad slot per segment), so the lanes of a
// segmented pass fall on distinct banks.  Each pass is a scan of affine maps:
//   d'_0 = d_0, d'_j = d_j + fr_j d'_{j-1};  w_{n-1} = ip_{n-1} d'_{n-1},
//   w_j = ip_j (d'_j + g_wl w_{j+1}).
__host__ __device__ inline int seg_lg(int n, int lanes)
{
    int lg = 0;
    while ((lanes << lg) < n) ++lg;
    return lg;
}
__device__ __forceinline__ int padj(int j, int lg) { return j + (j >> lg); }
__host__ __device__ inline int padded_len(int n, int lanes) { return n + (n >> seg_lg(n, lanes)) + 1; }

__device__ __forceinline__ void affine_compose(double& P, double& Q, double Pp, double Qp)
{
    Q = P * Qp + Q;          // x -> P (Pp x + Qp) + Q
    P = P * Pp;
}

template <int LANES>
__device__ __forceinline__ void tridiag_solve_lanes(double* __restrict__ d, const double* __restrict__ fr,
                                                    const double* __restrict__ ip, double gw, int n, int s,
                                                    int lg)
{
    const int j0 = s << lg, j1 = min(n, (s + 1) << lg);
    const int base = j0 + s;                 // padded index of j0
    double P = 1.0, Q = 0.0;
    for (int j = j0, p = base; j < j1; ++j, ++p) {
        Q = d[p] + fr[p] * Q;
        P = fr[p] * P;
    }
    for (int off = 1; off < LANES; off <<= 1) {
        const double Pp = __shfl_up(P, off, LANES), Qp = __shfl_up(Q, off, LANES);
        if (s >= off) affine_compose(P, Q, Pp, Qp);
    }
    double x = __shfl_up(Q, 1, LANES);
    if (s == 0) x = 0.0;
    for (int j = j0, p = base; j < j1; ++j, ++p) {
        x = d[p] + fr[p] * x;
        d[p] = x;
    }
    P = 1.0;
    Q = 0.0;
    for (int j = j1 - 1, p = base + (j1 - 1 - j0); j >= j0; --j, --p) {
        const double f = (j == n - 1) ? 0.0 : ip[p] * gw;
        Q = ip[p] * d[p] + f * Q;
        P = f * P;
    }
    for (int off = 1; off < LANES; off <<= 1) {
        const double Pp = __shfl_down(P, off, LANES), Qp = __shfl_down(Q, off, LANES);
        if (s + off < LANES) affine_compose(P, Q, Pp, Qp);
    }
    x = __shfl_down(Q, 1, LANES);
    if (s == LANES - 1) x = 0.0;
    for (int j = j1 - 1, p = base + (j1 - 1 - j0); j >= j0; --j, --p) {
        const double f = (j == n - 1) ? 0.0 : ip[p] * gw;
        x = ip[p] * d[p] + f * x;
        d[p] = x;
    }
}

// Stage the T_i coefficients of row i in padded LDS order.
__device__ __forceinline__ void stage_row_coeffs(double* sfr, double* sip, const double* fr,
                                                 const double* ip, int i, int n, int lg, int nthreads)
{
    for (int j = threadIdx.x; j < n; j += nthreads) {
        sfr[padj(j, lg)] = fr[(int64_t)i * n + j];
        sip[padj(j, lg)] = ip[(int64_t)i * n + j];
    }
}

// ---------------------------------------------------------------------------
template <typename T, int NT, bool IR, int W>
struct SweepCtx {
    using acc_t = typename Frag<T>::acc_t;
    static constexpr int n_p = 64 * NT;
    static constexpr int ldy = n_p + 4;
    static constexpr int TW = 4 * NT / W;    // row tiles per wave
    static constexpr int NTHR = 64 * W;
    static constexpr int LR = NTHR / 16;     // recovery lanes per input vector
    const SweepArgs& a;
    T* ybuf;
    T* Zs;
    const T* H;
    int w, l, q, col, b;
    bool bval;
    T g;
    double dmax = 0.0, umax = 0.0;   // refinement: largest correction and solution entry seen

    __device__ __forceinline__ int row_of(int t, int v) const { return 16 * (TW * w + t) + Frag<T>::drow(q, v); }
    __device__ __forceinline__ int64_t rowoff(int i) const { return ((int64_t)blockIdx.x * a.m + i) * 16 * n_p + col * n_p; }
    __device__ __forceinline__ T* zrow(int i) const { return Zs + (int64_t)i * 16 * n_p + col * n_p; }
    __device__ __forceinline__ double vin(int i) const { return bval ? a.V[(int64_t)b * a.m + i] : 0.0; }

    // panel <- f_i + g * (z terms); f_i = V_i c_i, or the residual panel R_i when refining
    __device__ __forceinline__ void set_panel(int i, const acc_t (&zacc)[TW], bool with_acc, int zrow_a, int zrow_b) {
        const bool from_r = IR && a.iter > 0;
        const double vb = from_r ? 0.0 : vin(i);
        const double* ci = a.c + (int64_t)i * n_p;
        const T* Ri = from_r ? reinterpret_cast<const T*>(a.R) + rowoff(i) : nullptr;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = row_of(t, v);
                T y = from_r ? (k < a.n ? Ri[pos<T>(k)] : (T)0) : (T)(ci[k] * vb);
                if (with_acc) y += g * zacc[t][v];
                if (zrow_a >= 0) y += g * zrow(zrow_a)[pos<T>(k)];
                if (zrow_b >= 0) y += g * zrow(zrow_b)[pos<T>(k)];
                ybuf[col * ldy + pos<T>(k)] = y;
            }
        __syncthreads();
    }
    __device__ __forceinline__ void put_panel(const acc_t (&u)[TW]) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) ybuf[col * ldy + pos<T>(row_of(t, v))] = u[t][v];
        __syncthreads();
    }
    __device__ __forceinline__ void store_z(int i, const acc_t (&z)[TW]) {
        T* zr = zrow(i);
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) zr[pos<T>(row_of(t, v))] = z[t][v];
    }
    // Word lines of row i from the bit-line voltages in the panel (LR lanes per
    // input vector), then both node voltages of the row go out in the paper's
    // interleaved order, coalesced.  wb: [16][padded n] + 2 padded coefficient rows.
    __device__ __forceinline__ void recover_row(int i, double* wb) {
        if (a.node_v == nullptr) return;
        const int n = a.n, cc = threadIdx.x / LR, s = threadIdx.x % LR;
        const int lg = seg_lg(n, LR), PL = padded_len(n, LR);
        double* sfr = wb + 16 * PL;
        double* sip = sfr + PL;
        stage_row_coeffs(sfr, sip, a.fr, a.ip, i, n, lg, NTHR);
        const int bb = 16 * (int)blockIdx.x + cc;
        const double* Gi = a.Gc + (int64_t)i * n;
        const double vb = (bb < a.B) ? a.V[(int64_t)bb * a.m + i] : 0.0;
        double* wv = wb + cc * PL;
        for (int j = s; j < n; j += LR)
            wv[padj(j, lg)] = Gi[j] * (double)ybuf[cc * ldy + pos<T>(j)] + (j == 0 ? a.g_src * vb : 0.0);
        __syncthreads();
        tridiag_solve_lanes<LR>(wv, sfr, sip, a.g_wl, n, s, lg);
        __syncthreads();
        const int two_n = 2 * n;
        const int64_t mn2 = (int64_t)2 * a.m * n;
        for (int c2 = 0; c2 < 16; ++c2) {          // one input vector at a time, coalesced
            const int b2 = 16 * (int)blockIdx.x + c2;
            if (b2 >= a.B) break;
            double* out = a.node_v + (int64_t)b2 * mn2 + (int64_t)i * two_n;
            for (int k = threadIdx.x; k < two_n; k += NTHR) {
                const int j = k >> 1;
                out[k] = (k & 1) ? (double)ybuf[c2 * ldy + pos<T>(j)] : wb[c2 * PL + padj(j, lg)];
            }
        }
    }
    // Row i of the back sweep is final in acc: emit the currents of row m-1, or (when
    // refining) add the correction to the float64 solution.
    __device__ __forceinline__ void settle(int i, const acc_t (&u)[TW]) {
        if (!IR) {
            if (i == a.m - 1) currents(u);
            return;
        }
        const int64_t ro = rowoff(i);
        const double* ui = a.Uin + ro;
        double* uo = a.Uout + ro;
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = pos<T>(row_of(t, v));
                const double d = (double)u[t][v];
                const double x = (a.iter > 0 ? ui[p] : 0.0) + d;
                uo[p] = x;
                dmax = fmax(dmax, fabs(d));
                umax = fmax(umax, fabs(x));
                if (i == a.m - 1) {
                    const int k = row_of(t, v);
                    if (bval && k < a.n) a.Iout[(int64_t)b * a.n + k] = a.g_sense * x;
                }
            }
    }
    // acc <- z_i + g * acc (back-sweep step)
    __device__ __forceinline__ void back_step(int i, acc_t (&acc)[TW]) {
        const T* zr = zrow(i);
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] = zr[pos<T>(row_of(t, v))] + g * acc[t][v];
    }
    __device__ __forceinline__ void currents(const acc_t (&u)[TW]) {
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = row_of(t, v);
                if (bval && k < a.n) a.Iout[(int64_t)b * a.n + k] = a.g_sense * (double)u[t][v];
            }
    }
    // Refinement bookkeeping for the slab: per input vector, stop when the error left after
    // this correction, estimated as |d| * min(1, |d| / |d_prev|), is <= tol * |u|.
    __device__ __forceinline__ void decide(double* red) {
        double dm = dmax, um = umax;
        for (int off = 16; off < 64; off <<= 1) {
            dm = fmax(dm, __shfl_xor(dm, off));
            um = fmax(um, __shfl_xor(um, off));
        }
        __syncthreads();
        if (l < 16) {
            red[w * 16 + l] = dm;
            red[16 * W + w * 16 + l] = um;
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            double D = 0.0, U = 0.0;
            for (int k = 0; k < W; ++k) {
                D = fmax(D, red[k * 16 + threadIdx.x]);
                U = fmax(U, red[16 * W + k * 16 + threadIdx.x]);
            }
            double* dprev = a.dnorm + (int64_t)blockIdx.x * 16 + threadIdx.x;
            const double est = (a.iter > 0 && *dprev > 0.0) ? D * fmin(1.0, D / *dprev) : D;
            const bool ok = (D == 0.0) || (a.iter > 0 && est <= a.tol * U);
            *dprev = D;
            const bool all = __all(ok) != 0;    // lanes 0..15 of wave 0 are the only active lanes
            if (threadIdx.x == 0) {
                const bool last = a.iter + 1 >= a.max_iter;
                if (all || last) {
                    a.slab_done[blockIdx.x] = 1;
                    a.slab_final[blockIdx.x] = (a.iter + 1) & 1;
                    atomicMax(a.flags + kIrIters, a.iter + 1);
                    if (!all) atomicOr(a.flags + kErrConv, 1);
                }
            }
        }
    }
};

template <int NT> struct SweepWaves { static constexpr int value = (NT % 2 == 0) ? 8 : 4; };

template <typename T, int NT, bool IR>
__global__ __launch_bounds__(64 * SweepWaves<NT>::value) void sweep_kernel(SweepArgs a)
{
    constexpr int W = SweepWaves<NT>::value;
    extern __shared__ __align__(32) unsigned char smem_raw[];
    using acc_t = typename Frag<T>::acc_t;
    using Ctx = SweepCtx<T, NT, IR, W>;
    constexpr int TW = Ctx::TW;
    if (IR && a.iter > 0 && a.slab_done[blockIdx.x]) return;
    const int m = a.m, kt = m / 2;
    const int l = threadIdx.x & 63;
    Ctx x{a, reinterpret_cast<T*>(smem_raw),
          reinterpret_cast<T*>(a.Z) + (int64_t)blockIdx.x * m * 16 * Ctx::n_p,
          reinterpret_cast<const T*>(a.H), (int)(threadIdx.x >> 6), l, l >> 4, l & 15,
          16 * (int)blockIdx.x + (l & 15), false, (T)a.g_bl};
    x.bval = x.b < a.B;
    const int64_t blk = (int64_t)Ctx::n_p * Ctx::n_p;
    double* wb = reinterpret_cast<double*>(smem_raw + 16 * Ctx::ldy * sizeof(T));
    acc_t acc[TW];
    // forward, top chain
    if (kt > 0) {
        x.set_panel(0, acc, false, -1, -1);
        for (int i = 0; i < kt; ++i) {
            panel_product<T, NT, TW>(acc, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.store_z(i, acc);
            if (i + 1 < kt) x.set_panel(i + 1, acc, true, -1, -1);
        }
    }
    // forward, bottom chain
    if (m - 1 > kt) {
        x.set_panel(m - 1, acc, false, -1, -1);
        for (int i = m - 1; i > kt; --i) {
            panel_product<T, NT, TW>(acc, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.store_z(i, acc);
            if (i - 1 > kt) x.set_panel(i - 1, acc, true, -1, -1);
        }
    }
    // twist row
    x.set_panel(kt, acc, false, kt > 0 ? kt - 1 : -1, kt + 1 < m ? kt + 1 : -1);
    panel_product<T, NT, TW>(acc, x.H + kt * blk, x.ybuf, Ctx::ldy, x.w, l);
    x.store_z(kt, acc);             // the downward back sweep restarts from this row
    x.settle(kt, acc);
    const bool fused = !IR && a.node_v != nullptr;
    if (fused) {
        x.put_panel(acc);
        x.recover_row(kt, wb);
    }
    // back, upward
    if (kt > 0) {
        if (!fused) x.put_panel(acc);
        for (int i = kt - 1; i >= 0; --i) {
            acc_t u[TW];
            panel_product<T, NT, TW>(u, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.back_step(i, u);
            x.settle(i, u);
            if (i > 0 || fused) x.put_panel(u);
            if (fused) x.recover_row(i, wb);
        }
    }
    // back, downward
    if (kt + 1 < m) {
        {
            const T* zr = x.zrow(kt);
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[t][v] = zr[pos<T>(x.row_of(t, v))];
        }
        x.put_panel(acc);
        for (int i = kt + 1; i < m; ++i) {
            panel_product<T, NT, TW>(acc, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.back_step(i, acc);
            x.settle(i, acc);
            if (i < m - 1 || fused) x.put_panel(acc);
            if (fused) x.recover_row(i, wb);
        }
    }
    if (IR) x.decide(wb);
}

// ---------------------------------------------------------------------------
// Residual of the condensed system for the refinement, in float64:
//   r_i = V_i c_i - (E_i u_i - g_bl (u_{i-1} + u_{i+1})),
//   E_i u_i = Q_i u_i - Gam_i T_i^{-1} (Gam_i u_i)
// with T_i^{-1} applied by the same Thomas recurrences as the word-line
// recovery; rounded to float for the correction sweep.  One workgroup per
// (row, 8 input vectors), 32 lanes per vector.
constexpr int kResCols = 8;
constexpr int kResLanes = 32;

__global__ __launch_bounds__(256) void residual_kernel(ResidualArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = a.n, m = a.m, n_p = a.n_p;
    const int i = blockIdx.y;
    const int slab = blockIdx.x / 2, half = blockIdx.x % 2;
    if (a.slab_done[slab]) return;
    const int lg = seg_lg(n, kResLanes), PL = padded_len(n, kResLanes);
    double* wb = reinterpret_cast<double*>(smem_raw);             // [kResCols][PL]
    double* sfr = wb + kResCols * PL;
    double* sip = sfr + PL;
    stage_row_coeffs(sfr, sip, a.fr, a.ip, i, n, lg, 256);
    const int c = threadIdx.x / kResLanes, s = threadIdx.x % kResLanes;
    const int colg = half * kResCols + c;
    const int b = 16 * slab + colg;
    const double* Gi = a.Gc + (int64_t)i * n;
    const double* Ui = a.U + (((int64_t)slab * m + i) * 16 + colg) * n_p;
    double* w = wb + c * PL;
    for (int j = s; j < n; j += kResLanes) w[padj(j, lg)] = Gi[j] * Ui[j];
    __syncthreads();
    tridiag_solve_lanes<kResLanes>(w, sfr, sip, a.g_wl, n, s, lg);
    __syncthreads();
    const double vb = (b < a.B) ? a.V[(int64_t)b * m + i] : 0.0;
    const double* ci = a.c + (int64_t)i * n_p;
    const double* qi = a.q + (int64_t)i * n;
    const double* Uup = (i > 0) ? Ui - 16 * (int64_t)n_p : nullptr;
    const double* Udn = (i + 1 < m) ? Ui + 16 * (int64_t)n_p : nullptr;
    float* Ri = reinterpret_cast<float*>(a.R) + (((int64_t)slab * m + i) * 16 + colg) * n_p;
    for (int j = s; j < n; j += kResLanes) {
        double r = ci[j] * vb - (qi[j] * Ui[j] - Gi[j] * w[padj(j, lg)]);
        if (Uup) r += a.g_bl * Uup[j];
        if (Udn) r += a.g_bl * Udn[j];
        Ri[j] = (float)r;
    }
    for (int j = n + s; j < n_p; j += kResLanes) Ri[j] = 0.0f;      // padding stays zero
}

// Word-line recovery and node-voltage output from the float64 solution of the
// refinement (one workgroup per (row, 8 input vectors), 32 lanes per vector).
constexpr int kRecCols = kResCols;

template <typename T>
__global__ __launch_bounds__(256) void recover_kernel(RecoverArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = a.n, m = a.m, n_p = a.n_p;
    const int lg = seg_lg(n, kResLanes), PL = padded_len(n, kResLanes);
    double* ub = reinterpret_cast<double*>(smem_raw);       // [kRecCols][n]
    double* wb = ub + kRecCols * n;                           // [kRecCols][PL]
    double* sfr = wb + kRecCols * PL;
    double* sip = sfr + PL;
    const int i = blockIdx.y;
    const int slab = blockIdx.x / 2, half = blockIdx.x % 2;
    stage_row_coeffs(sfr, sip, a.fr, a.ip, i, n, lg, 256);
    const int c = threadIdx.x / kResLanes, s = threadIdx.x % kResLanes;
    const int b = 16 * slab + half * kRecCols + c;
    if (a.slab_final != nullptr) {
        const double* Ui = a.U[a.slab_final[slab]] + ((int64_t)slab * m + i) * 16 * n_p;
        for (int e = threadIdx.x; e < kRecCols * n; e += blockDim.x) {
            const int cc = e / n, j = e % n;
            ub[e] = Ui[(half * kRecCols + cc) * n_p + pos<T>(j)];
        }
    } else {
        const T* Zi = reinterpret_cast<const T*>(a.Z) + ((int64_t)slab * m + i) * 16 * n_p;
        for (int e = threadIdx.x; e < kRecCols * n; e += blockDim.x) {
            const int cc = e / n, j = e % n;
            ub[e] = (double)Zi[(half * kRecCols + cc) * n_p + pos<T>(j)];
        }
    }
    __syncthreads();
    const double* Gi = a.Gc + (int64_t)i * n;
    const double vin = (b < a.B) ? a.V[(int64_t)b * m + i] : 0.0;
    const double* u = ub + c * n;
    double* wv = wb + c * PL;
    for (int j = s; j < n; j += kResLanes) wv[padj(j, lg)] = Gi[j] * u[j] + (j == 0 ? a.g_src * vin : 0.0);
    __syncthreads();
    tridiag_solve_lanes<kResLanes>(wv, sfr, sip, a.g_wl, n, s, lg);
    __syncthreads();
    if (a.node_v == nullptr) return;
    for (int cc = 0; cc < kRecCols; ++cc) {
        const int bb = 16 * slab + half * kRecCols + cc;
        if (bb >= a.B) break;
        double* out = a.node_v + (int64_t)bb * 2 * m * n + (int64_t)2 * i * n;
        for (int k = threadIdx.x; k < 2 * n; k += blockDim.x) {
            const int j = k >> 1;
            out[k] = (k & 1) ? ub[cc * n + j] : wb[cc * PL + padj(j, lg)];
        }
    }
}

// ---------------------------------------------------------------------------
template <typename T, int NT, bool IR>
hipError_t launch_sweep_nt(const SweepArgs& a, hipStream_t s)
{
    constexpr int W = SweepWaves<NT>::value;
    const size_t panel = 16 * (size_t)(64 * NT + 4) * sizeof(T);
    const size_t extra = IR ? 2 * 16 * W * sizeof(double)
                            : (16 + 2) * (size_t)padded_len(a.n, 4 * W) * sizeof(double);
    hipLaunchKernelGGL((sweep_kernel<T, NT, IR>), dim3(a.nslab), dim3(64 * W), panel + extra, s, a);
    return hipGetLastError();
}

template <typename T, bool IR>
hipError_t launch_sweep(const SweepArgs& a, hipStream_t s)
{
    switch (a.n_p / 64) {
        case 1: return launch_sweep_nt<T, 1, IR>(a, s);
        case 2: return launch_sweep_nt<T, 2, IR>(a, s);
        case 3: return launch_sweep_nt<T, 3, IR>(a, s);
        case 4: return launch_sweep_nt<T, 4, IR>(a, s);
        case 5: return launch_sweep_nt<T, 5, IR>(a, s);
        case 6: return launch_sweep_nt<T, 6, IR>(a, s);
        case 7: return launch_sweep_nt<T, 7, IR>(a, s);
        case 8: return launch_sweep_nt<T, 8, IR>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace xbk

hipError_t xbk_launch_sweep(const xbk::SweepArgs& a, bool fp32, hipStream_t s)
{
    return fp32 ? xbk::launch_sweep<float, false>(a, s) : xbk::launch_sweep<double, false>(a, s);
}

hipError_t xbk_launch_sweep_ir(const xbk::SweepArgs& a, hipStream_t s)
{
    return xbk::launch_sweep<float, true>(a, s);
}

hipError_t xbk_launch_residual(const xbk::ResidualArgs& a, hipStream_t s)
{
    const size_t lds = ((size_t)xbk::kResCols + 2) * xbk::padded_len(a.n, xbk::kResLanes) * sizeof(double);
    hipLaunchKernelGGL(xbk::residual_kernel, dim3(2 * a.nslab, a.m), dim3(256), lds, s, a);
    return hipGetLastError();
}

hipError_t xbk_launch_recover(const xbk::RecoverArgs& a, bool fp32, hipStream_t s)
{
    const size_t lds = (xbk::kRecCols * (size_t)a.n +
                        (xbk::kRecCols + 2) * (size_t)xbk::padded_len(a.n, xbk::kResLanes)) * sizeof(double);
    dim3 grid(2 * a.nslab, a.m);
    if (fp32)
        hipLaunchKernelGGL(xbk::recover_kernel<float>, grid, dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(xbk::recover_kernel<double>, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

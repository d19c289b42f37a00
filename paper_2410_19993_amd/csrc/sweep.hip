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
// them for the whole sweep: no grid synchronisation at all, and no thread
// reads another's global writes, so barriers order LDS only.  Per row block
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
// H_i is FRG, the panel is [column][CPR position].  The chunks of H stream
// through a ring of DP register sets: chunk K + DP is requested as soon as
// chunk K has been issued to the matrix cores, so DP chunks are always in
// flight (the loop is unrolled by DP to keep the ring indices static).  The
// ring runs on across row blocks: on entry it holds the first DP chunks of Hi,
// and the last DP chunks of Hi are followed by the first DP of Hnext, so the
// next row's loads are in flight during the barriers and bookkeeping between
// products.
template <typename T> struct SweepRing { static constexpr int value = sizeof(T) == 8 ? 2 : 4; };

template <typename T, int NT, int TW>
struct HRing {
    using v4 = typename Vec4<T>::type;
    static constexpr int DP = SweepRing<T>::value;
    v4 r[DP][TW];
    __device__ __forceinline__ void prime(const T* __restrict__ Hi, int w, int l) {
#pragma unroll
        for (int d = 0; d < DP; ++d)
#pragma unroll
            for (int t = 0; t < TW; ++t) r[d][t] = load_frag<T>(Hi, 4 * NT, TW * w + t, d, l);
    }
};

struct NoHook {
    __device__ __forceinline__ void operator()(int) const {}
};

// hook(K) runs after the products of chunk K have been issued (K is a
// compile-time constant once the loop is unrolled), so that independent
// work can fill the matrix-core loop.
template <typename T, int NT, int TW, typename Hook>
__device__ __forceinline__ void panel_product(typename Frag<T>::acc_t (&acc)[TW], HRing<T, NT, TW>& ring,
                                              const T* __restrict__ Hi, const T* __restrict__ Hnext,
                                              const T* ybuf, int ldy, int w, int l, const Hook& hook)
{
    using v4 = typename Vec4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    constexpr int n_p = 64 * NT;
    constexpr int KC = n_p / 16;
    constexpr int DP = SweepRing<T>::value;
    static_assert(KC % DP == 0, "chunk count must be a multiple of the ring depth");
    const int q = l >> 4, r = l & 15;
#pragma unroll
    for (int t = 0; t < TW; ++t) acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int K0 = 0; K0 < KC; K0 += DP) {
#pragma unroll
        for (int d = 0; d < DP; ++d) {
            const int K = K0 + d;
            const v4 bv = *reinterpret_cast<const v4*>(ybuf + r * ldy + 16 * K + 4 * q);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < TW; ++t) acc[t] = Frag<T>::mma(ring.r[d][t][s], bv[s], acc[t]);
            if (K + DP < KC) {
#pragma unroll
                for (int t = 0; t < TW; ++t) ring.r[d][t] = load_frag<T>(Hi, KC, TW * w + t, K + DP, l);
            } else {
#pragma unroll
                for (int t = 0; t < TW; ++t) ring.r[d][t] = load_frag<T>(Hnext, KC, TW * w + t, K + DP - KC, l);
            }
            hook(K);
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

// Order this wave's LDS writes before later LDS reads of other lanes of the
// same wave (no workgroup barrier needed: the data is private to the wave).
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

typedef double d2_t __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Per-workgroup state of a sweep.  Global inputs of a step (right-hand-side
// rows, forward results z_i, row coefficients of the word-line recovery) are
// requested before the step's product and consumed after it, so their latency
// hides behind the matrix cores.
//
// Word-line recovery (float64 sweep with node voltages): wave w recovers the
// VW input vectors w*VW.. of the slab, LR lanes each, in a buffer private to
// the wave; only the staging of the row coefficients is shared.  The node
// voltages of a recovered row are written during the next row's product, one
// 16-byte store per lane every few K chunks, so the stores spread over the
// whole sweep instead of bursting between products.
template <typename T, int NT, bool IR, int W>
struct SweepCtx {
    using acc_t = typename Frag<T>::acc_t;
    static constexpr int n_p = 64 * NT;
    static constexpr int ldy = n_p + 4;
    static constexpr int TW = 4 * NT / W;    // row tiles per wave
    static constexpr int NTHR = 64 * W;
    static constexpr int VW = 16 / W;        // input vectors a wave recovers
    static constexpr int LR = 64 / VW;       // lanes per input vector in the recovery
    static constexpr int CPT = (n_p + NTHR - 1) / NTHR;   // row coefficients per thread
    static constexpr int NST = VW * NT;      // node-voltage stores per lane and row
    const SweepArgs& a;
    T* ybuf;          // [16][ldy] right-hand side / solution panel
    double* wv;       // [VW][PL] this wave's word-line buffers
    double* coef;     // [3][PL] fr, ip, G of the row being recovered
    T* Zs;
    const T* H;
    int w, l, q, col, b;
    bool bval;
    T g;
    int lg = 0, PL = 0;                      // recovery segment width (log2), padded row length
    double dmax = 0.0, umax = 0.0;           // refinement: largest correction and solution entry
    double pf_fr[CPT], pf_ip[CPT], pf_g[CPT], pf_v = 0.0;

    // Lane (q, col) of wave w holds rows row_of(t, v) of tile t, item v.  In panel
    // (CPR) order those rows sit at poff + 16 t + v, so every panel access is a
    // wave-uniform base, one per-lane offset and a small constant.
    __device__ __forceinline__ int row_of(int t, int v) const { return 16 * (TW * w + t) + Frag<T>::drow(q, v); }
    __device__ __forceinline__ uint32_t poff() const { return (uint32_t)(16 * TW * w + 4 * q); }
    __device__ __forceinline__ uint32_t lane_off() const { return (uint32_t)(col * n_p) + poff(); }
    __device__ __forceinline__ int64_t slab_row(int i) const { return ((int64_t)blockIdx.x * a.m + i) * 16 * n_p; }
    __device__ __forceinline__ T* zbase(int i) const { return Zs + (int64_t)i * 16 * n_p; }
    __device__ __forceinline__ T* zrow(int i) const { return zbase(i) + col * n_p; }
    __device__ __forceinline__ double vin(int i) const { return bval ? a.V[(int64_t)b * a.m + i] : 0.0; }

    // ---- forward sweep
    // this lane's rows of the right-hand side of row block i: V_i c_i, or the residual R_i
    __device__ __forceinline__ void load_rhs(int i, T (&f)[TW][4]) const {
        if (IR && a.iter > 0) {
            const T* Ri = reinterpret_cast<const T*>(a.R) + slab_row(i);
            const uint32_t o = lane_off();
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) f[t][v] = row_of(t, v) < a.n ? Ri[o + 16 * t + v] : (T)0;
        } else {
            const double vb = vin(i);
            const double* ci = a.c + (int64_t)i * n_p;         // zero on the padding
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) f[t][v] = (T)(ci[row_of(t, v)] * vb);
        }
    }
    // panel <- f + g * zacc (+ g * the forward results of rows zrow_a, zrow_b: the twist)
    __device__ __forceinline__ void set_panel(const T (&f)[TW][4], const acc_t (&zacc)[TW], bool with_acc,
                                              int zrow_a, int zrow_b) {
        lds_barrier();
        const uint32_t o = lane_off(), lo = (uint32_t)(col * ldy) + poff();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T y = f[t][v];
                if (with_acc) y += g * zacc[t][v];
                if (zrow_a >= 0) y += g * zbase(zrow_a)[o + 16 * t + v];
                if (zrow_b >= 0) y += g * zbase(zrow_b)[o + 16 * t + v];
                ybuf[lo + 16 * t + v] = y;
            }
        lds_barrier();
    }
    __device__ __forceinline__ void store_z(int i, const acc_t (&z)[TW]) {
        T* zr = zbase(i);
        const uint32_t o = lane_off();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) zr[o + 16 * t + v] = z[t][v];
    }

    // ---- back sweep
    __device__ __forceinline__ void load_z(int i, T (&zp)[TW][4]) const {
        const T* zr = zbase(i);
        const uint32_t o = lane_off();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) zp[t][v] = zr[o + 16 * t + v];
    }
    // refinement: the float64 solution before this sweep (zero at the first sweep)
    __device__ __forceinline__ void load_u(int i, double (&up)[TW][4]) const {
        const double* ui = a.Uin + slab_row(i);
        const uint32_t o = lane_off();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) up[t][v] = (IR && a.iter > 0) ? ui[o + 16 * t + v] : 0.0;
    }
    // acc <- z_i + g * acc
    __device__ __forceinline__ void back_step(const T (&zp)[TW][4], acc_t (&acc)[TW]) const {
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] = zp[t][v] + g * acc[t][v];
    }
    // panel <- u (and, when recovering, the staged coefficients of the row)
    __device__ __forceinline__ void put_panel(const acc_t (&u)[TW], bool commit) {
        lds_barrier();
        const uint32_t lo = (uint32_t)(col * ldy) + poff();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) ybuf[lo + 16 * t + v] = u[t][v];
        if (commit) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int j = (int)threadIdx.x + c * NTHR;
                if (j < a.n) {
                    const int p = padj(j, lg);
                    coef[p] = pf_fr[c];
                    coef[PL + p] = pf_ip[c];
                    coef[2 * PL + p] = pf_g[c];
                }
            }
        }
        lds_barrier();
    }
    // Row i of the back sweep is final in u: emit the currents of row m-1, or (when
    // refining) add the correction to the float64 solution.
    __device__ __forceinline__ void settle(int i, const acc_t (&u)[TW], const double (&up)[TW][4]) {
        if (!IR) {
            if (i == a.m - 1) currents(u);
            return;
        }
        double* uo = a.Uout + slab_row(i);
        const uint32_t o = lane_off();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double d = (double)u[t][v];
                const double x = up[t][v] + d;
                uo[o + 16 * t + v] = x;
                dmax = fmax(dmax, fabs(d));
                umax = fmax(umax, fabs(x));
                if (i == a.m - 1) {
                    const int k = row_of(t, v);
                    if (bval && k < a.n) a.Iout[(int64_t)b * a.n + k] = a.g_sense * x;
                }
            }
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

    // ---- word-line recovery: T_i w_i = g_src V_i e_0 + Gam_i u_i
    // request row i's coefficients and this lane's input (staged by put_panel)
    __device__ __forceinline__ void prefetch_row(int i) {
        const int64_t o = (int64_t)i * a.n;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int jj = min((int)threadIdx.x + c * NTHR, a.n - 1);
            pf_fr[c] = a.fr[o + jj];
            pf_ip[c] = a.ip[o + jj];
            pf_g[c] = a.Gc[o + jj];
        }
        const int bb = 16 * (int)blockIdx.x + w * VW + l / LR;
        pf_v = (bb < a.B) ? a.V[(int64_t)bb * a.m + i] : 0.0;
    }
    // word lines of the row whose bit-line voltages are in the panel, for this wave's vectors
    __device__ __forceinline__ void solve_row() {
        const int n = a.n, v = l / LR, s = l % LR, cc = w * VW + v;
        double* wr = wv + v * PL;
        for (int j = s; j < n; j += LR)
            wr[padj(j, lg)] = coef[2 * PL + padj(j, lg)] * (double)ybuf[cc * ldy + pos<T>(j)] +
                              (j == 0 ? a.g_src * pf_v : 0.0);
        wave_lds_fence();
        tridiag_solve_lanes<LR>(wr, coef, coef + PL, a.g_wl, n, s, lg);
        wave_lds_fence();
    }
    // k-th node-voltage store of recovered row i (i < 0: none): the pair (w_j, u_j) of
    // this wave's vector k / NT, j = 64 (k % NT) + lane, in the interleaved node order.
    // The lane-dependent addresses are rebuilt from an opaque copy of the lane index,
    // so the compiler cannot hoist all NST of them out of the row loop into registers.
    __device__ __forceinline__ void out_store(int i, int k) const {
        const int v = k / NT, cc = w * VW + v;
        const int bb = 16 * (int)blockIdx.x + cc;              // wave-uniform
        if (i < 0 || bb >= a.B) return;
        int lane = l;
        asm volatile("" : "+v"(lane));
        const int j = 64 * (k % NT) + lane;
        if (j >= a.n) return;
        const double wj = wv[v * PL + padj(j, lg)];
        const double uj = (double)ybuf[cc * ldy + pos<T>(j)];
        double* base = a.node_v + ((int64_t)bb * a.m + i) * 2 * a.n;
        *reinterpret_cast<d2_t*>(base + 2 * j) = d2_t{wj, uj};
    }
    __device__ __forceinline__ void out_row(int i) const {
#pragma unroll
        for (int k = 0; k < NST; ++k) out_store(i, k);
    }

    // Refinement bookkeeping for the slab: per input vector, stop when the error left after
    // this correction, estimated as |d| * min(1, |d| / |d_prev|), is <= tol * |u|.
    __device__ __forceinline__ void decide(double* red) {
        double dm = dmax, um = umax;
        for (int off = 16; off < 64; off <<= 1) {
            dm = fmax(dm, __shfl_xor(dm, off));
            um = fmax(um, __shfl_xor(um, off));
        }
        lds_barrier();
        if (l < 16) {
            red[w * 16 + l] = dm;
            red[16 * W + w * 16 + l] = um;
        }
        lds_barrier();
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

// Node-voltage stores of a recovered row, spread over the K chunks of a product.
template <typename Ctx>
struct OutHook {
    const Ctx& x;
    int row;
    __device__ __forceinline__ void operator()(int K) const {
        constexpr int STEP = Ctx::n_p / 16 / Ctx::NST;
        if ((K + 1) % STEP == 0) {
            // keep each store's loads in place: hoisted together they would
            // hold every pending store's data in registers during the product
            __builtin_amdgcn_sched_barrier(0);
            x.out_store(row, K / STEP);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
};

template <int NT> struct SweepWaves { static constexpr int value = (NT % 2 == 0) ? 8 : 4; };

// LDS bytes of a sweep: panel, then either the word-line buffers and row coefficients
// (recovery) or the refinement's reduction scratch.
template <typename T, int NT, bool IR>
__host__ __device__ inline size_t sweep_lds_bytes(int n)
{
    constexpr int W = SweepWaves<NT>::value;
    const size_t panel = 16 * (size_t)(64 * NT + 4) * sizeof(T);
    const size_t extra = IR ? 2 * 16 * W * sizeof(double)
                            : (16 + 3) * (size_t)padded_len(n, 64 / (16 / W)) * sizeof(double);
    return panel + extra;
}

template <typename T, int NT, bool IR, bool REC>
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
    Ctx x{a, reinterpret_cast<T*>(smem_raw), nullptr, nullptr,
          reinterpret_cast<T*>(a.Z) + (int64_t)blockIdx.x * m * 16 * Ctx::n_p,
          reinterpret_cast<const T*>(a.H), __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), l, l >> 4, l & 15,
          16 * (int)blockIdx.x + (l & 15), false, (T)a.g_bl};
    x.bval = x.b < a.B;
    x.lg = seg_lg(a.n, Ctx::LR);
    x.PL = padded_len(a.n, Ctx::LR);
    double* extra = reinterpret_cast<double*>(smem_raw + 16 * Ctx::ldy * sizeof(T));
    x.wv = extra + x.w * Ctx::VW * x.PL;
    x.coef = extra + 16 * x.PL;
    const int64_t blk = (int64_t)Ctx::n_p * Ctx::n_p;
    auto Hb = [&](int i) { return x.H + i * blk; };
    acc_t acc[TW];
    T f[TW][4];
    const NoHook none{};
    // H blocks in sweep order: 0..kt-1, m-1..kt+1, kt, kt-1..0, kt+1..m-1
    HRing<T, NT, TW> ring;
    ring.prime(Hb(kt > 0 ? 0 : (m - 1 > kt ? m - 1 : kt)), x.w, l);
    // forward, top chain
    if (kt > 0) {
        x.load_rhs(0, f);
        x.set_panel(f, acc, false, -1, -1);
        for (int i = 0; i < kt; ++i) {
            if (i + 1 < kt) x.load_rhs(i + 1, f);
            const int nx = i + 1 < kt ? i + 1 : (m - 1 > kt ? m - 1 : kt);
            panel_product<T, NT, TW>(acc, ring, Hb(i), Hb(nx), x.ybuf, Ctx::ldy, x.w, l, none);
            x.store_z(i, acc);
            if (i + 1 < kt) x.set_panel(f, acc, true, -1, -1);
        }
    }
    // forward, bottom chain
    if (m - 1 > kt) {
        x.load_rhs(m - 1, f);
        x.set_panel(f, acc, false, -1, -1);
        for (int i = m - 1; i > kt; --i) {
            if (i - 1 > kt) x.load_rhs(i - 1, f);
            panel_product<T, NT, TW>(acc, ring, Hb(i), Hb(i - 1 > kt ? i - 1 : kt), x.ybuf, Ctx::ldy, x.w, l, none);
            x.store_z(i, acc);
            if (i - 1 > kt) x.set_panel(f, acc, true, -1, -1);
        }
    }
    // twist row
    double up[TW][4];
    x.load_rhs(kt, f);
    x.set_panel(f, acc, false, kt > 0 ? kt - 1 : -1, kt + 1 < m ? kt + 1 : -1);
    x.load_u(kt, up);
    if (REC) x.prefetch_row(kt);
    panel_product<T, NT, TW>(acc, ring, Hb(kt), Hb(kt > 0 ? kt - 1 : (kt + 1 < m ? kt + 1 : kt)), x.ybuf, Ctx::ldy,
                             x.w, l, none);
    x.store_z(kt, acc);             // the downward back sweep restarts from this row
    x.settle(kt, acc, up);
    int pend = -1;                  // recovered row whose node voltages are not yet written
    if (REC) {
        x.put_panel(acc, true);
        x.solve_row();
        pend = kt;
    }
    // back, upward
    if (kt > 0) {
        if (!REC) x.put_panel(acc, false);
        for (int i = kt - 1; i >= 0; --i) {
            T zp[TW][4];
            x.load_z(i, zp);
            x.load_u(i, up);
            acc_t u[TW];
            const T* Hn = Hb(i > 0 ? i - 1 : (kt + 1 < m ? kt + 1 : i));
            if (REC) {
                x.prefetch_row(i);
                panel_product<T, NT, TW>(u, ring, Hb(i), Hn, x.ybuf, Ctx::ldy, x.w, l, OutHook<Ctx>{x, pend});
            } else {
                panel_product<T, NT, TW>(u, ring, Hb(i), Hn, x.ybuf, Ctx::ldy, x.w, l, none);
            }
            x.back_step(zp, u);
            x.settle(i, u, up);
            if (REC) {
                x.put_panel(u, true);
                x.solve_row();
                pend = i;
            } else if (i > 0) {
                x.put_panel(u, false);
            }
        }
    }
    // back, downward
    if (kt + 1 < m) {
        if (REC && pend >= 0) {
            x.out_row(pend);        // the panel is about to be reset to u_kt
            pend = -1;
        }
        {
            T zp[TW][4];
            x.load_z(kt, zp);
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[t][v] = zp[t][v];
        }
        x.put_panel(acc, false);
        for (int i = kt + 1; i < m; ++i) {
            T zp[TW][4];
            x.load_z(i, zp);
            x.load_u(i, up);
            const T* Hn = Hb(i + 1 < m ? i + 1 : i);
            if (REC) {
                x.prefetch_row(i);
                panel_product<T, NT, TW>(acc, ring, Hb(i), Hn, x.ybuf, Ctx::ldy, x.w, l, OutHook<Ctx>{x, pend});
            } else {
                panel_product<T, NT, TW>(acc, ring, Hb(i), Hn, x.ybuf, Ctx::ldy, x.w, l, none);
            }
            x.back_step(zp, acc);
            x.settle(i, acc, up);
            if (REC) {
                x.put_panel(acc, true);
                x.solve_row();
                pend = i;
            } else if (i < m - 1) {
                x.put_panel(acc, false);
            }
        }
    }
    if (REC && pend >= 0) x.out_row(pend);
    if (IR) x.decide(extra);
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
    lds_barrier();
    tridiag_solve_lanes<kResLanes>(w, sfr, sip, a.g_wl, n, s, lg);
    lds_barrier();
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
    lds_barrier();
    const double* Gi = a.Gc + (int64_t)i * n;
    const double vin = (b < a.B) ? a.V[(int64_t)b * m + i] : 0.0;
    const double* u = ub + c * n;
    double* wv = wb + c * PL;
    for (int j = s; j < n; j += kResLanes) wv[padj(j, lg)] = Gi[j] * u[j] + (j == 0 ? a.g_src * vin : 0.0);
    lds_barrier();
    tridiag_solve_lanes<kResLanes>(wv, sfr, sip, a.g_wl, n, s, lg);
    lds_barrier();
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
    const size_t lds = sweep_lds_bytes<T, NT, IR>(a.n);
    if constexpr (!IR) {
        if (a.node_v != nullptr) {
            hipLaunchKernelGGL((sweep_kernel<T, NT, IR, true>), dim3(a.nslab), dim3(64 * W), lds, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((sweep_kernel<T, NT, IR, false>), dim3(a.nslab), dim3(64 * W), lds, s, a);
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

hipError_t xbk_launch_sweep(const xbk::SweepArgs& a, hipStream_t s)
{
    return xbk::launch_sweep<double, false>(a, s);
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

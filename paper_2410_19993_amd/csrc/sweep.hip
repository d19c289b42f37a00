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
#include "xbar.h"

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
constexpr int kRing = 2;        // chunk-sets of H in flight per wave

// Matrix-core waves per workgroup: 8 for even n_p / 64 (n_p / 128 row tiles each);
// for odd n_p / 64 either n_p / 64 waves of 4 tiles or (n_p = 320) 4 waves of 5
// tiles, whichever keeps the accumulators and the H ring without spills next to
// the helper waves.
template <int NT> struct SweepWaves { static constexpr int value = (NT % 2 == 0) ? 8 : (NT == 5 ? 4 : NT); };
// The refinement sweeps keep two panels, so that a row's panel update needs one
// barrier: the panel written is the one the product before the previous barrier read.
template <bool IR> struct SweepPanels { static constexpr int value = IR ? 2 : 1; };

template <typename T, int NT, int TW, int DP>
struct HRing {
    using v4 = typename Vec4<T>::type;
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
template <typename T, int NT, int TW, int DP, typename Hook>
__device__ __forceinline__ void panel_product(typename Frag<T>::acc_t (&acc)[TW], HRing<T, NT, TW, DP>& ring,
                                              const T* __restrict__ Hi, const T* __restrict__ Hnext,
                                              const T* ybuf, int ldy, int w, int l, const Hook& hook)
{
    using v4 = typename Vec4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    constexpr int n_p = 64 * NT;
    constexpr int KC = n_p / 16;
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
            // chunk K + DP: of this block, or of the next one (one load site, a selected
            // block pointer: the float64 waves need the registers this saves)
            const T* Hl = K + DP < KC ? Hi : Hnext;
            const int cn = K + DP < KC ? K + DP : K + DP - KC;
            if constexpr (sizeof(T) == 4) {
                // float32: tile by tile, the tile's products and then the load of its
                // chunk K + DP, with a scheduling fence after every second tile, so that
                // the loads stay spread between the products (the float64 waves have no
                // registers to spare for this ordering)
#pragma unroll
                for (int t = 0; t < TW; ++t) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[t] = Frag<T>::mma(ring.r[d][t][s], bv[s], acc[t]);
                    ring.r[d][t] = load_frag<T>(Hl, KC, TW * w + t, cn, l);
                    if (t & 1) __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int t = 0; t < TW; ++t) acc[t] = Frag<T>::mma(ring.r[d][t][s], bv[s], acc[t]);
#pragma unroll
                for (int t = 0; t < TW; ++t) ring.r[d][t] = load_frag<T>(Hl, KC, TW * w + t, cn, l);
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
// smallest power of two >= x
constexpr int seg_cap(int x) { return x <= 1 ? 1 : 2 * seg_cap((x + 1) / 2); }

__device__ __forceinline__ void affine_compose(double& P, double& Q, double Pp, double Qp)
{
    Q = P * Qp + Q;          // x -> P (Pp x + Qp) + Q
    P = P * Pp;
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
// Per-workgroup state of a sweep, as seen by the matrix-core waves.  Global
// inputs of a step (right-hand-side rows, and in the refinement sweeps the
// forward results z_i and the float64 solution) are requested before the
// step's product and consumed after it, so their latency hides behind the
// matrix cores.
template <typename T, int NT, bool IR, int W>
struct SweepCtx {
    using acc_t = typename Frag<T>::acc_t;
    static constexpr int n_p = 64 * NT;
    static constexpr int ldy = n_p + 4;
    static constexpr int TW = 4 * NT / W;    // row tiles per wave
    static constexpr bool DB = SweepPanels<IR>::value == 2;
    const SweepArgs& a;
    T* ybuf;          // [16][ldy] right-hand side / solution panel
    T* Zs;
    const T* H;
    int w, l, q, col, b;
    bool bval;
    T g;
    double dmax = 0.0, umax = 0.0;           // refinement: largest correction and solution entry
    double dbad = 0.0;                       // 0, or NaN once a correction entry was not finite
    T* yalt = nullptr;                       // two panels: the one the next update writes

    // Lane (q, col) of wave w holds rows row_of(t, v) of tile t, item v.  In panel
    // (CPR) order those rows sit at poff + 16 t + v, so every panel access is a
    // wave-uniform base, one per-lane offset and a small constant.
    __device__ __forceinline__ int row_of(int t, int v) const { return 16 * (TW * w + t) + Frag<T>::drow(q, v); }
    __device__ __forceinline__ uint32_t poff() const { return (uint32_t)(16 * TW * w + 4 * q); }
    __device__ __forceinline__ uint32_t lane_off() const { return (uint32_t)(col * n_p) + poff(); }
    __device__ __forceinline__ int64_t slab_row(int i) const { return ((int64_t)a.slab * a.m + i) * 16 * n_p; }
    __device__ __forceinline__ T* zbase(int i) const { return Zs + (int64_t)i * 16 * n_p; }
    __device__ __forceinline__ double vin(int i) const {
        return bval ? (a.unit ? (b == i ? 1.0 : 0.0) : a.V[(int64_t)b * a.m + i]) : 0.0;
    }

    // ---- forward sweep
    // this lane's rows of the right-hand side of row block i: V_i c_i, or the residual R_i.
    // LAST = false: i is known not to be the last row (the loads inside the chains,
    // which overlap a product and must not add to its registers).
    template <bool LAST = true>
    __device__ __forceinline__ void load_rhs(int i, T (&f)[TW][4]) const {
        if (IR && a.iter > 0) {
            const T* Ri = reinterpret_cast<const T*>(a.R) + slab_row(i);
            const uint32_t o = lane_off();
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) f[t][v] = row_of(t, v) < a.n ? Ri[o + 16 * t + v] : (T)0;
        } else if (a.term) {
            // reciprocal ordering: g_sense V[b][n-1-k] at the last row only (clamped
            // indices keep every load in bounds)
            const double* Vb = a.V + (int64_t)(bval ? b : 0) * a.n + (a.n - 1);
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) f[t][v] = (T)0;
            if (LAST && i == a.m - 1) {
#pragma unroll
                for (int t = 0; t < TW; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int k = row_of(t, v);
                        const double x = Vb[-min(k, a.n - 1)];
                        f[t][v] = (T)((bval && k < a.n) ? a.g_sense * x : 0.0);
                    }
            }
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
        // one panel: wait until every wave has read it; two: the other one was last
        // read by the product before the previous barrier
        if (!DB) lds_barrier();
        T* dst = DB ? yalt : ybuf;
        const uint32_t o = lane_off(), lo = (uint32_t)(col * ldy) + poff();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T y = f[t][v];
                if (with_acc) y += g * zacc[t][v];
                if (zrow_a >= 0) y += g * zbase(zrow_a)[o + 16 * t + v];
                if (zrow_b >= 0) y += g * zbase(zrow_b)[o + 16 * t + v];
                dst[lo + 16 * t + v] = y;
            }
        lds_barrier();
        if (DB) {
            yalt = ybuf;
            ybuf = dst;
        }
    }
    // z_i is read back only in the back sweep: streamed past L2 so that it does not
    // displace the H blocks the workgroups share
    __device__ __forceinline__ void store_z(int i, const acc_t (&z)[TW]) {
        T* zr = zbase(i);
        const uint32_t o = lane_off();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) __builtin_nontemporal_store(z[t][v], zr + o + 16 * t + v);
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
    // panel <- u
    __device__ __forceinline__ void put_panel(const acc_t (&u)[TW]) {
        if (!DB) lds_barrier();
        T* dst = DB ? yalt : ybuf;
        const uint32_t lo = (uint32_t)(col * ldy) + poff();
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[lo + 16 * t + v] = u[t][v];
        lds_barrier();
        if (DB) {
            yalt = ybuf;
            ybuf = dst;
        }
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
                dbad += d * 0.0;             // one instruction; fmax alone would drop a NaN
                umax = fmax(umax, fabs(x));
                if (i == a.m - 1) {
                    const int k = row_of(t, v);
                    if (bval && k < a.n) a.Iout[(int64_t)b * a.n + k] = a.g_sense * x;
                }
            }
    }
    __device__ __forceinline__ void currents(const acc_t (&u)[TW]) {
        const bool bad = a.tile_bad != nullptr && *a.tile_bad != 0;     // batches: a spoilt crossbar
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = row_of(t, v);
                if (bval && k < a.n) a.Iout[(int64_t)b * a.n + k] = bad ? NAN : a.g_sense * (double)u[t][v];
            }
    }

    // Refinement bookkeeping for the slab: per input vector, stop when the error left after
    // this correction, estimated as |d| * min(1, |d| / |d_prev|), is <= tol * |u|.
    __device__ __forceinline__ void decide(double* red) {
        double dm = dmax + dbad, um = umax;
        for (int off = 16; off < 64; off <<= 1) {
            dm = nan_max(dm, __shfl_xor(dm, off));
            um = nan_max(um, __shfl_xor(um, off));
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
                D = nan_max(D, red[k * 16 + threadIdx.x]);
                U = nan_max(U, red[16 * W + k * 16 + threadIdx.x]);
            }
            double* dprev = a.dnorm + (int64_t)a.slab * 16 + threadIdx.x;
            const double est = (a.iter > 0 && *dprev > 0.0) ? D * fmin(1.0, D / *dprev) : D;
            const bool ok = (D == 0.0) || (a.iter > 0 && est <= a.tol * U);
            *dprev = D;
            const bool all = __all(ok) != 0;    // lanes 0..15 of wave 0 are the only active lanes
            if (threadIdx.x == 0) {
                const bool last = a.iter + 1 >= a.max_iter;
                if (all || last) {
                    a.slab_done[a.slab] = 1;
                    a.slab_final[a.slab] = (a.iter + 1) & 1;
                    atomicMax(a.flags + kIrIters, a.iter + 1);
                    if (!all) atomicOr(a.flags + kErrConv, 1);
                }
            }
        }
    }
};

constexpr int kHelpers = 4;      // helper waves of the float64 sweep (one per SIMD)
// The refinement sweeps recover no word lines and have no helper waves: their
// matrix-core waves pull the H blocks into L2 themselves (measured faster than
// helpers doing it, at two waves per SIMD instead of three).
template <bool IR> struct SweepHelpers { static constexpr int value = IR ? 0 : kHelpers; };

// Pull this workgroup's share of an H block into L2 with WAVES waves: one 4-byte
// load per 128-byte line.  The loads are issued before the work they overlap and
// their values consumed after it, so no wave waits on them.  A single crossbar's
// slabs (workgroups b, b + 8, ... on one XCD) take 1/32 of the block each; in a
// batch a crossbar's slabs share one XCD and take 1/16 each.
template <typename T, int NT, int WAVES>
struct L2Pull {
    static constexpr size_t LINE = 128;
    static constexpr size_t STEP = (size_t)WAVES * 64 * LINE;
    static constexpr size_t BLK = (size_t)(64 * NT) * (64 * NT) * sizeof(T);
    static constexpr size_t SHARE = ((BLK / 32) + LINE - 1) & ~(LINE - 1);
    static constexpr size_t SHARE_B = ((BLK / 16) + LINE - 1) & ~(LINE - 1);
    static constexpr int IT = (int)((SHARE_B + STEP - 1) / STEP);
    uint32_t pv[IT];
    uint32_t keep = 0;                        // xor of the pulled words (kept live)
    __device__ __forceinline__ void issue(const SweepArgs& a, const T* blk, int wv, int l) {
        const char* p = reinterpret_cast<const char*>(blk);
        const bool batched = a.batch > 1;
        const size_t share = batched ? SHARE_B : SHARE;
        const size_t lo = batched ? SHARE_B * ((size_t)a.slab & 15) : SHARE * (((size_t)blockIdx.x >> 3) & 31);
        const size_t hi = min(BLK, lo + share);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const size_t off = lo + ((size_t)it * WAVES + wv) * 64 * LINE + LINE * (size_t)l;
            pv[it] = (blk != nullptr && off < hi) ? *reinterpret_cast<const uint32_t*>(p + off) : 0u;
        }
    }
    __device__ __forceinline__ void consume() {
#pragma unroll
        for (int it = 0; it < IT; ++it) keep ^= pv[it];
    }
    // a store that never happens but keeps the loads
    __device__ __forceinline__ void retire(const SweepArgs& a, int l) const {
        if (keep == 0x9e3779b9u) a.sink[l] = (double)keep;
    }
};

// ---------------------------------------------------------------------------
// Schedule of the float64 sweep as pairs of workgroup barriers (a panel update
// each).  The matrix-core waves pass them as set_panel / put_panel calls; the
// helper waves count them off with the same enumeration:
//   pairs 0 .. kt-1          forward, top chain: product of row p follows
//   pairs kt .. F-1          forward, bottom chain: rows m-1 .. kt+1
//   pair  F                  twist: row kt
//   pair  F+1                panel <- u_kt; then rows kt-1 .. 0 (one pair after each)
//   pair  F+2+kt             (kt+1 < m) panel <- z_kt, restart; then rows kt+1 .. m-1
// with F = kt + max(0, m-1-kt).  Without the upward back sweep (up = false: only
// the output currents, which depend on u_{m-1} alone, are wanted) rows kt+1 .. m-1
// follow pair F+1 directly: the panel already holds u_kt.
struct SweepPlan {
    int m, kt, F;
    bool up;
    __device__ __forceinline__ SweepPlan(int m_, bool up_)
        : m(m_), kt(m_ / 2), F(m_ / 2 + max(0, m_ - 1 - m_ / 2)), up(up_) {}
    __device__ __forceinline__ int pairs() const {
        const int down = m - 1 - kt;               // rows kt+1 .. m-1
        return up ? F + 2 + kt + (down > 0 ? 1 + down : 0) : F + 2 + down;
    }
    // row whose product follows pair p (-1: none)
    __device__ __forceinline__ int product_after(int p) const {
        if (p < kt) return p;
        if (p < F) return m - 1 - (p - kt);
        if (p == F) return kt;
        int q = p - (F + 1);                       // 0: panel <- u_kt, then u_{kt-1}, ...
        if (!up) return kt + 1 + q < m ? kt + 1 + q : -1;
        if (q <= kt) {
            const int i = kt - q;                  // panel holds u_i
            return i > 0 ? i - 1 : -1;
        }
        q -= kt + 1;
        if (kt + 1 < m) return q == 0 ? kt + 1 : (kt + q + 1 < m ? kt + q + 1 : -1);
        return -1;
    }
    // row whose bit-line voltages are in the panel after pair p, to recover (-1: none)
    __device__ __forceinline__ int recover_after(int p) const {
        if (p <= F || !up) return -1;
        int q = p - (F + 1);
        if (q <= kt) return kt - q;
        q -= kt + 1;
        return (kt + 1 < m && q > 0) ? kt + q : -1;
    }
};

// Helper waves of the float64 sweep.  While the matrix-core waves run the product
// that follows a barrier pair, the helpers
//  * pull this workgroup's share of the next row's H block into L2 (workgroups b,
//    b+8, ... share an L2; each takes 1/32 of the block), so that the products
//    find H in L2 instead of missing all together at the same addresses;
//  * in the back sweep, recover the word lines of the row whose bit lines are in
//    the panel,
//        T_i w_i = g_src V_i e_0 + Gam_i u_i,
//    writing that row's node voltages in the paper's interleaved order.  Helper
//    wave h takes input vectors 4h .. 4h+3, 16 lanes each, every lane a contiguous
//    segment of the row; the T_i coefficients are read from L2.
template <typename T, int NT>
struct SweepHelper {
    static constexpr int n_p = 64 * NT;
    static constexpr int ldy = n_p + 4;
    static constexpr int LR = 16;             // lanes per input vector
    static constexpr int VPW = 64 / LR;       // input vectors per helper wave
    const SweepArgs& a;
    const T* ybuf;
    double* wv;                               // [16][PL] word-line buffers
    int h, l, lg, PL;
    L2Pull<T, NT, kHelpers> pull;             // this workgroup's share of the next H block
    // Row coefficients of T_i (fr, ip) and the devices G of the row recovered after the
    // next barrier pair: requested at the start of a task, written to the free half of
    // the double-buffered LDS copy at its end, published by the next barrier pair.
    static constexpr int HT = kHelpers * 64;                 // helper threads
    static constexpr int CPT = (n_p + HT - 1) / HT;          // coefficients per thread
    double* coef;                                            // [2][3][PL]
    double cf[CPT], ci[CPT], cg[CPT];
    double vnext = 0.0, vcur = 0.0;                          // input V of this lane's vector
    __device__ __forceinline__ void stage_load(int i) {
        const int64_t o = (int64_t)i * a.n;
        const int bb = 16 * a.slab + h * VPW + l / LR;
        vnext = (bb < a.B && !a.unit && !a.term) ? a.V[(int64_t)bb * a.m + i] : 0.0;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int jj = min(h * 64 + l + c * HT, a.n - 1);
            cf[c] = a.fr[o + jj];
            ci[c] = a.ip[o + jj];
            cg[c] = a.Gc[o + jj];
        }
    }
    __device__ __forceinline__ void stage_store(int buf) {
        vcur = vnext;
        double* cb = coef + buf * 3 * PL;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int j = h * 64 + l + c * HT;
            if (j < a.n) {
                const int pj = padj(j, lg);
                cb[pj] = cf[c];
                cb[PL + pj] = ci[c];
                cb[2 * PL + pj] = cg[c];
            }
        }
    }
    // Word lines and node voltages of row i for this wave's vectors, from the staged
    // coefficients in buffer buf.  Loops run to compile-time bounds with masked lanes.
    static constexpr int KJ = (n_p + LR - 1) / LR;          // j's per lane in the first pass
    static constexpr int SEG = seg_cap(KJ);                  // longest lane segment
    __device__ __forceinline__ void recover(int i, int buf) {
        const int n = a.n, v = l / LR, s = l % LR, cc = h * VPW + v;
        const int bb = 16 * a.slab + cc;
        const double* fr = coef + buf * 3 * PL;              // padded like d
        const double* ip = fr + PL;
        const double* Gi = fr + 2 * PL;
        const double vb = vcur;
        double* d = wv + cc * PL;
        const int spare = PL - 1;                              // never a padded index of j < n
#pragma unroll 8
        for (int k = 0; k < KJ; ++k) {
            const int j = s + LR * k;
            const bool ok = j < n;
            const int pj = padj(ok ? j : n - 1, lg);
            const double val = Gi[pj] * (double)ybuf[cc * ldy + pos<T>(ok ? j : n - 1)] +
                               (j == 0 ? a.g_src * vb : 0.0);
            d[ok ? pj : spare] = val;
        }
        wave_lds_fence();
        // T_i w = d by forward and backward affine scans over the LR lanes of a vector
        const int j0 = s << lg, len = max(0, min(n - j0, 1 << lg)), base = j0 + s;
        const double gw = a.g_wl;
        double P = 1.0, Q = 0.0;
#pragma unroll 8
        for (int e = 0; e < SEG; ++e) {
            const bool ok = e < len;
            const int p = ok ? base + e : spare;
            const double f = ok ? fr[p] : 0.0;               // fr at j = 0 is zero
            const double Qn = d[p] + f * Q, Pn = f * P;
            Q = ok ? Qn : Q;
            P = ok ? Pn : P;
        }
        for (int off = 1; off < LR; off <<= 1) {
            const double Pp = __shfl_up(P, off, LR), Qp = __shfl_up(Q, off, LR);
            if (s >= off) affine_compose(P, Q, Pp, Qp);
        }
        double x = __shfl_up(Q, 1, LR);
        if (s == 0) x = 0.0;
#pragma unroll 8
        for (int e = 0; e < SEG; ++e) {
            const bool ok = e < len;
            const int p = ok ? base + e : spare;
            const double f = ok ? fr[p] : 0.0;
            const double xn = d[p] + f * x;
            x = ok ? xn : x;
            d[p] = x;
        }
        P = 1.0;
        Q = 0.0;
#pragma unroll 8
        for (int e = SEG - 1; e >= 0; --e) {
            const bool ok = e < len;
            const int p = ok ? base + e : spare;
            const double ipj = ok ? ip[p] : 0.0;
            const double f = (j0 + e >= n - 1) ? 0.0 : ipj * gw;
            const double Qn = ipj * d[p] + f * Q, Pn = f * P;
            Q = ok ? Qn : Q;
            P = ok ? Pn : P;
        }
        for (int off = 1; off < LR; off <<= 1) {
            const double Pp = __shfl_down(P, off, LR), Qp = __shfl_down(Q, off, LR);
            if (s + off < LR) affine_compose(P, Q, Pp, Qp);
        }
        x = __shfl_down(Q, 1, LR);
        if (s == LR - 1) x = 0.0;
#pragma unroll 8
        for (int e = SEG - 1; e >= 0; --e) {
            const bool ok = e < len;
            const int p = ok ? base + e : spare;
            const double ipj = ok ? ip[p] : 0.0;
            const double f = (j0 + e >= n - 1) ? 0.0 : ipj * gw;
            const double xn = ipj * d[p] + f * x;
            x = ok ? xn : x;
            d[p] = x;
        }
        wave_lds_fence();
        // node voltages (w_j, u_j) of the wave's vectors, 1 KB per store instruction
        typedef double d2v __attribute__((ext_vector_type(2)));
        for (int vv = 0; vv < VPW; ++vv) {
            const int c2 = h * VPW + vv, b2 = 16 * a.slab + c2;
            if (b2 >= a.B) break;
            double* out = a.node_v + ((int64_t)b2 * a.m + i) * 2 * n;
#pragma unroll 4
            for (int k = 0; k < NT; ++k) {
                const int j = 64 * k + l;
                if (j < n)
                    __builtin_nontemporal_store(d2v{wv[c2 * PL + padj(j, lg)], (double)ybuf[c2 * ldy + pos<T>(j)]},
                                                reinterpret_cast<d2v*>(out + 2 * j));
            }
        }
    }
    // the whole schedule, one barrier pair at a time
    __device__ void run(bool rec, bool up) {
        const SweepPlan sp(a.m, up);
        const int np = sp.pairs();
        const T* H = reinterpret_cast<const T*>(a.H);
        for (int p = 0; p < np; ++p) {
            lds_barrier();
            lds_barrier();
            const int rn = rec && p + 1 < np ? sp.recover_after(p + 1) : -1;
            if (rn >= 0) stage_load(rn);
            // during the product after pair p: the block of the next product
            int nb = sp.product_after(p + 1);
            if (nb < 0 && p + 2 < np) nb = sp.product_after(p + 2);
            pull.issue(a, nb >= 0 ? H + (int64_t)nb * n_p * n_p : nullptr, h, l);
            const int r = sp.recover_after(p);
            if (rec && r >= 0) recover(r, p & 1);
            pull.consume();
            if (rn >= 0) stage_store((p + 1) & 1);
        }
        pull.retire(a, l);
    }
};

// LDS bytes of a sweep: the panel, then the word-line buffers and two copies of
// the row coefficients (float64 sweep) or the refinement's reduction scratch.
template <typename T, int NT, bool IR>
__host__ __device__ inline size_t sweep_lds_bytes(int n)
{
    constexpr int W = SweepWaves<NT>::value;
    const size_t panel = SweepPanels<IR>::value * 16 * (size_t)(64 * NT + 4) * sizeof(T);
    const size_t extra = IR ? 2 * 16 * W * sizeof(double)
                            : (16 + 2 * 3) * (size_t)padded_len(n, SweepHelper<T, NT>::LR) * sizeof(double);
    return panel + extra;
}

// Workgroup -> (crossbar, slab) of a batch: workgroup b runs on XCD b % 8, and the
// slabs of crossbar t all get the XCD t % 8, so they share its L2 for the H blocks.
// Returns false for the padding workgroups past the last crossbar.
template <typename T, int NT>
__device__ __forceinline__ bool batch_slab(SweepArgs& a)
{
    if (a.batch <= 1) {
        a.slab = blockIdx.x;
        return true;
    }
    const int S = a.slabs_per, xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int t = (local / S) * 8 + xcd;
    if (t >= a.batch) return false;
    a.slab = local % S;
    const int64_t n_p = 64 * NT;
    a.H = reinterpret_cast<const T*>(a.H) + (int64_t)t * a.m * n_p * n_p;
    a.c += (int64_t)t * a.m * n_p;
    if (!a.unit) a.V += (int64_t)t * a.B * a.m;
    a.Z = reinterpret_cast<T*>(a.Z) + (int64_t)t * S * a.m * 16 * n_p;
    a.Iout += (int64_t)t * a.B * a.n;
    if (a.tile_bad) a.tile_bad += t;
    return true;
}

template <typename T, int NT, bool IR, bool REC>
__global__ __launch_bounds__(64 * (SweepWaves<NT>::value + SweepHelpers<IR>::value)) void sweep_kernel(SweepArgs a)
{
    constexpr int W = SweepWaves<NT>::value;
    constexpr int NH = SweepHelpers<IR>::value;
    constexpr int DP = kRing;
    extern __shared__ __align__(32) unsigned char smem_raw[];
    using acc_t = typename Frag<T>::acc_t;
    using Ctx = SweepCtx<T, NT, IR, W>;
    constexpr int TW = Ctx::TW;
    if (!batch_slab<T, NT>(a)) return;
    if (IR && a.iter > 0 && a.slab_done[a.slab]) return;
    const int m = a.m, kt = m / 2;
    const int l = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    double* extra = reinterpret_cast<double*>(smem_raw + SweepPanels<IR>::value * 16 * Ctx::ldy * sizeof(T));
    if constexpr (NH > 0) {
        if (wave >= W) {
            // helper waves (float64 sweep): word-line recovery and the H pulls
            const int PL = padded_len(a.n, SweepHelper<T, NT>::LR);
            SweepHelper<T, NT> hp{a, reinterpret_cast<const T*>(smem_raw), extra, wave - W, l,
                                   seg_lg(a.n, SweepHelper<T, NT>::LR), PL};
            hp.coef = extra + 16 * PL;
            // the helpers' latency-bound work gets issue priority over the matrix-core
            // waves, which have independent work queued behind every instruction
            __builtin_amdgcn_s_setprio(3);
            hp.run(REC, REC);
            return;
        }
    }
    Ctx x{a, reinterpret_cast<T*>(smem_raw),
          reinterpret_cast<T*>(a.Z) + (int64_t)a.slab * m * 16 * Ctx::n_p,
          reinterpret_cast<const T*>(a.H), wave, l, l >> 4, l & 15,
          16 * a.slab + (l & 15), false, (T)a.g_bl};
    x.bval = x.b < a.B;
    if constexpr (Ctx::DB) x.yalt = x.ybuf + 16 * Ctx::ldy;
    const int64_t blk = (int64_t)Ctx::n_p * Ctx::n_p;
    auto Hb = [&](int i) { return x.H + i * blk; };
    acc_t acc[TW];
    T f[TW][4];
    const NoHook none{};
    // H blocks in sweep order: 0..kt-1, m-1..kt+1, kt, kt-1..0, kt+1..m-1
    HRing<T, NT, TW, DP> ring;
    ring.prime(Hb(kt > 0 ? 0 : (m - 1 > kt ? m - 1 : kt)), x.w, l);
    // the product of row i; block nx follows it.  Without helper waves, the share of
    // block nx is pulled into L2 during the product.
    L2Pull<T, NT, W> pull;
    auto product = [&](acc_t (&out)[TW], int i, int nx) {
        if constexpr (NH == 0) pull.issue(a, Hb(nx), x.w, l);
        panel_product<T, NT, TW>(out, ring, Hb(i), Hb(nx), x.ybuf, Ctx::ldy, x.w, l, none);
        if constexpr (NH == 0) pull.consume();
    };
    // forward, top chain
    if (kt > 0) {
        x.load_rhs(0, f);
        x.set_panel(f, acc, false, -1, -1);
        for (int i = 0; i < kt; ++i) {
            if (i + 1 < kt) x.template load_rhs<false>(i + 1, f);
            const int nx = i + 1 < kt ? i + 1 : (m - 1 > kt ? m - 1 : kt);
            product(acc, i, nx);
            x.store_z(i, acc);
            if (i + 1 < kt) x.set_panel(f, acc, true, -1, -1);
        }
    }
    // forward, bottom chain
    if (m - 1 > kt) {
        x.load_rhs(m - 1, f);
        x.set_panel(f, acc, false, -1, -1);
        for (int i = m - 1; i > kt; --i) {
            if (i - 1 > kt) x.template load_rhs<false>(i - 1, f);
            product(acc, i, i - 1 > kt ? i - 1 : kt);
            x.store_z(i, acc);
            if (i - 1 > kt) x.set_panel(f, acc, true, -1, -1);
        }
    }
    // twist row.  Only the output currents wanted (float64, no node voltages): they
    // depend on u_{m-1} alone, so the upward back sweep is skipped.
    constexpr bool UP = IR || REC;
    double up[TW][4];
    x.load_rhs(kt, f);
    x.set_panel(f, acc, false, kt > 0 ? kt - 1 : -1, kt + 1 < m ? kt + 1 : -1);
    x.load_u(kt, up);
    const int after_twist = (UP && kt > 0) ? kt - 1 : (kt + 1 < m ? kt + 1 : kt);
    product(acc, kt, after_twist);
    if (UP) x.store_z(kt, acc);     // the downward back sweep restarts from this row
    x.settle(kt, acc, up);
    x.put_panel(acc);
    // back, upward
    if (UP) {
        for (int i = kt - 1; i >= 0; --i) {
            T zp[TW][4];
            if (IR) x.load_z(i, zp);    // refinement sweeps: no helpers, request z before the product
            x.load_u(i, up);
            acc_t u[TW];
            product(u, i, i > 0 ? i - 1 : (kt + 1 < m ? kt + 1 : i));
            if (!IR) x.load_z(i, zp);   // float64 sweep: after the product (no registers to spare in it)
            x.back_step(zp, u);
            x.settle(i, u, up);
            x.put_panel(u);
        }
    }
    // back, downward
    if (kt + 1 < m) {
        if (UP) {
            T zp[TW][4];
            x.load_z(kt, zp);
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[t][v] = zp[t][v];
            x.put_panel(acc);
        }
        for (int i = kt + 1; i < m; ++i) {
            T zp[TW][4];
            if (IR) x.load_z(i, zp);
            x.load_u(i, up);
            product(acc, i, i + 1 < m ? i + 1 : i);
            if (!IR) x.load_z(i, zp);
            x.back_step(zp, acc);
            x.settle(i, acc, up);
            x.put_panel(acc);
        }
    }
    if (IR && a.tol >= 0.0) x.decide(extra);
    if constexpr (NH == 0) pull.retire(a, l);
}

// ---------------------------------------------------------------------------
// T_i w = d for one input vector over LANES lanes (padded LDS vectors d, fr, ip as
// above), with loops run to the compile-time bound SEG >= 1 << lg and masked lanes
// (they touch only the spare slot), so that each pass's LDS loads issue ahead of
// its recurrence.  FULL: every lane owns exactly SEG elements (n = LANES * SEG),
// so no lane is masked and the LDS offsets are immediates.
template <int LANES, int SEG, bool FULL>
__device__ __forceinline__ void tridiag_solve_masked(double* __restrict__ d, const double* __restrict__ fr,
                                                     const double* __restrict__ ip, double gw, int n, int s,
                                                     int lg, int spare)
{
    const int j0 = s << lg, len = FULL ? SEG : max(0, min(n - j0, 1 << lg)), base = j0 + s;
    double P = 1.0, Q = 0.0;
#pragma unroll 8
    for (int e = 0; e < SEG; ++e) {
        const bool ok = FULL || e < len;
        const int p = ok ? base + e : spare;
        const double f = ok ? fr[p] : 0.0;                   // fr at j = 0 is zero
        const double Qn = d[p] + f * Q, Pn = f * P;
        Q = ok ? Qn : Q;
        P = ok ? Pn : P;
    }
    for (int off = 1; off < LANES; off <<= 1) {
        const double Pp = __shfl_up(P, off, LANES), Qp = __shfl_up(Q, off, LANES);
        if (s >= off) affine_compose(P, Q, Pp, Qp);
    }
    double x = __shfl_up(Q, 1, LANES);
    if (s == 0) x = 0.0;
#pragma unroll 8
    for (int e = 0; e < SEG; ++e) {
        const bool ok = FULL || e < len;
        const int p = ok ? base + e : spare;
        const double f = ok ? fr[p] : 0.0;
        const double xn = d[p] + f * x;
        x = ok ? xn : x;
        d[p] = x;
    }
    P = 1.0;
    Q = 0.0;
#pragma unroll 8
    for (int e = SEG - 1; e >= 0; --e) {
        const bool ok = FULL || e < len;
        const int p = ok ? base + e : spare;
        const double ipj = ok ? ip[p] : 0.0;
        const double f = (j0 + e >= n - 1) ? 0.0 : ipj * gw;
        const double Qn = ipj * d[p] + f * Q, Pn = f * P;
        Q = ok ? Qn : Q;
        P = ok ? Pn : P;
    }
    for (int off = 1; off < LANES; off <<= 1) {
        const double Pp = __shfl_down(P, off, LANES), Qp = __shfl_down(Q, off, LANES);
        if (s + off < LANES) affine_compose(P, Q, Pp, Qp);
    }
    x = __shfl_down(Q, 1, LANES);
    if (s == LANES - 1) x = 0.0;
#pragma unroll 8
    for (int e = SEG - 1; e >= 0; --e) {
        const bool ok = FULL || e < len;
        const int p = ok ? base + e : spare;
        const double ipj = ok ? ip[p] : 0.0;
        const double f = (j0 + e >= n - 1) ? 0.0 : ipj * gw;
        const double xn = ipj * d[p] + f * x;
        x = ok ? xn : x;
        d[p] = x;
    }
}

// Row walkers of the refinement: one workgroup per half slab (8 input vectors,
// 32 lanes each) walks the rows i = 0..m-1, so that every row of the float64
// solution is read from memory once (a lane keeps elements j = s + 32k of the
// rows it still needs in registers).  The next row of the solution and of the
// coefficients is requested before a row's tridiagonal solve, so that its
// latency hides behind it; the coefficients pass through double-buffered LDS.  One workgroup barrier per
// row publishes the next row's coefficients.
constexpr int kRwCols = 8;                                  // input vectors per workgroup
constexpr int kRwLanes = 32;                                // lanes per input vector
constexpr int kRwJ = (XBAR_MAX_N + kRwLanes - 1) / kRwLanes;   // elements per lane
constexpr int kRwSeg = seg_cap(kRwJ);                       // longest lane segment of a solve
constexpr int kRwCoef = (XBAR_MAX_N + 255) / 256;           // staged coefficients per thread and array

template <int NC>
struct RowCoeffs {
    double r[NC][kRwCoef];
    // arrays [m][ld] of row i, element j of thread t at j = t + 256 k
    __device__ __forceinline__ void load(const double* const (&src)[NC], const int (&ld)[NC], int i, int n) {
#pragma unroll
        for (int k = 0; k < kRwCoef; ++k) {
            const int jj = min((int)threadIdx.x + 256 * k, n - 1);
#pragma unroll
            for (int q = 0; q < NC; ++q) r[q][k] = src[q][(int64_t)i * ld[q] + jj];
        }
    }
    __device__ __forceinline__ void store(double* cb, int PL, int n, int lg) const {
#pragma unroll
        for (int k = 0; k < kRwCoef; ++k) {
            const int j = threadIdx.x + 256 * k;
            if (j < n) {
                const int pj = padj(j, lg);
#pragma unroll
                for (int q = 0; q < NC; ++q) cb[q * PL + pj] = r[q][k];
            }
        }
    }
};

__device__ __forceinline__ void rw_load_row(const double* __restrict__ Ui, int n, int s, double (&u)[kRwJ])
{
#pragma unroll
    for (int k = 0; k < kRwJ; ++k) {
        const int j = s + kRwLanes * k;
        u[k] = j < n ? Ui[j] : 0.0;
    }
}

// Residual of the condensed system for the refinement, in float64:
//   r_i = V_i c_i - (E_i u_i - g_bl (u_{i-1} + u_{i+1})),
//   E_i u_i = Q_i u_i - Gam_i T_i^{-1} (Gam_i u_i)
// with T_i^{-1} applied by the same Thomas recurrences as the word-line
// recovery; rounded to float for the correction sweep.
template <bool FULL>
__device__ __forceinline__ void residual_walk(const ResidualArgs& a, unsigned char* smem_raw)
{
    const int n = a.n, m = a.m, n_p = a.n_p;
    const int slab = blockIdx.x >> 1, half = blockIdx.x & 1;
    const int lg = seg_lg(n, kRwLanes), PL = padded_len(n, kRwLanes), spare = PL - 1;
    double* wb = reinterpret_cast<double*>(smem_raw);        // [8][PL] right-hand sides / solutions
    double* cb = wb + kRwCols * PL;                           // [2][5][PL] fr, ip, G, c, q of a row
    const int c = threadIdx.x / kRwLanes, s = threadIdx.x % kRwLanes;
    const int colg = half * kRwCols + c, b = 16 * slab + colg;
    const int64_t rs = 16 * (int64_t)n_p;
    const double* U = a.U + ((int64_t)slab * m * 16 + colg) * n_p;
    float* R = reinterpret_cast<float*>(a.R) + ((int64_t)slab * m * 16 + colg) * n_p;
    double* Rd = a.Rd ? a.Rd + ((int64_t)slab * m * 16 + colg) * n_p : nullptr;
    double* w = wb + c * PL;
    const double* const src[5] = {a.fr, a.ip, a.Gc, a.c, a.q};
    const int ld[5] = {n, n, n, n_p, n};
    RowCoeffs<5> rc;
    double up[kRwJ], uc[kRwJ];
#pragma unroll
    for (int k = 0; k < kRwJ; ++k) up[k] = 0.0;
    rw_load_row(U, n, s, uc);
    rc.load(src, ld, 0, n);
    rc.store(cb, PL, n, lg);
    __syncthreads();
    for (int i = 0; i < m; ++i) {
        const double* cf = cb + (i & 1) * 5 * PL;
        // the next row of the solution and of the coefficients, requested before
        // this row's solve and used after it
        double un[kRwJ];
#pragma unroll
        for (int k = 0; k < kRwJ; ++k) un[k] = 0.0;
        if (i + 1 < m) {
            rw_load_row(U + (i + 1) * rs, n, s, un);
            rc.load(src, ld, i + 1, n);
        }
        const double vb = (b < a.B && !a.matvec && !a.term) ? a.V[(int64_t)b * m + i] : 0.0;
        // reciprocal ordering: the terminations' right-hand side at the last row
        const double* Vt = (a.term && !a.matvec && b < a.B && i == m - 1) ? a.V + (int64_t)b * n : nullptr;
#pragma unroll
        for (int k = 0; k < kRwJ; ++k) {
            const int j = s + kRwLanes * k;
            if (FULL || j < n) w[padj(j, lg)] = cf[2 * PL + padj(j, lg)] * uc[k];
        }
        wave_lds_fence();
        tridiag_solve_masked<kRwLanes, kRwSeg, FULL>(w, cf, cf + PL, a.g_wl, n, s, lg, spare);
        wave_lds_fence();
        float* Ri = R + i * rs;
        double* Rdi = Rd ? Rd + i * rs : nullptr;
#pragma unroll
        for (int k = 0; k < kRwJ; ++k) {
            const int j = s + kRwLanes * k;
            if (FULL || j < n) {
                const int pj = padj(j, lg);
                // A u = E_i u_i - g_bl (u_{i-1} + u_{i+1}); the residual is V c - A u
                const double eu = cf[4 * PL + pj] * uc[k] - cf[2 * PL + pj] * w[pj];
                const double rhs = Vt ? a.g_sense * Vt[n - 1 - j] : cf[3 * PL + pj] * vb;
                const double r = a.matvec ? eu - a.g_bl * (up[k] + un[k]) : rhs - eu + a.g_bl * (up[k] + un[k]);
                if (Rdi)
                    Rdi[j] = r;
                else
                    Ri[j] = (float)r;
            }
        }
        for (int j = n + s; j < n_p; j += kRwLanes) {                 // padding stays zero
            if (Rdi)
                Rdi[j] = 0.0;
            else
                Ri[j] = 0.0f;
        }
        if (i + 1 < m) rc.store(cb + ((i + 1) & 1) * 5 * PL, PL, n, lg);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRwJ; ++k) {
            up[k] = uc[k];
            uc[k] = un[k];
        }
    }
}

__global__ __launch_bounds__(256) void residual_kernel(ResidualArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (a.slab_done[blockIdx.x >> 1]) return;
    if (a.n == kRwLanes * kRwSeg)
        residual_walk<true>(a, smem_raw);
    else
        residual_walk<false>(a, smem_raw);
}

// Word-line recovery and node-voltage output from the final float64 solution of
// the refinement: T_i w_i = g_src V_i e_0 + Gam_i u_i, then (w_ij, u_ij) in the
// paper's interleaved order, 16 bytes per lane and 512 contiguous bytes per vector
// and store instruction.
template <bool FULL>
__device__ __forceinline__ void recover_walk(const RecoverArgs& a, unsigned char* smem_raw)
{
    const int n = a.n, m = a.m, n_p = a.n_p;
    const int slab = blockIdx.x >> 1, half = blockIdx.x & 1;
    const int lg = seg_lg(n, kRwLanes), PL = padded_len(n, kRwLanes), spare = PL - 1;
    double* wb = reinterpret_cast<double*>(smem_raw);        // [8][PL]
    double* cb = wb + kRwCols * PL;                           // [2][3][PL] fr, ip, G of a row
    const int c = threadIdx.x / kRwLanes, s = threadIdx.x % kRwLanes;
    const int colg = half * kRwCols + c, b = 16 * slab + colg;
    const bool bval = b < a.B;
    const int64_t rs = 16 * (int64_t)n_p;
    const double* U = a.U[a.slab_final[slab]] + ((int64_t)slab * m * 16 + colg) * n_p;
    double* w = wb + c * PL;
    const double* const src[3] = {a.fr, a.ip, a.Gc};
    const int ld[3] = {n, n, n};
    RowCoeffs<3> rc;
    double uc[kRwJ];
    rw_load_row(U, n, s, uc);
    rc.load(src, ld, 0, n);
    rc.store(cb, PL, n, lg);
    __syncthreads();
    typedef double d2v __attribute__((ext_vector_type(2)));
    for (int i = 0; i < m; ++i) {
        const double* cf = cb + (i & 1) * 3 * PL;
        double un[kRwJ];
#pragma unroll
        for (int k = 0; k < kRwJ; ++k) un[k] = 0.0;
        if (i + 1 < m) {
            rw_load_row(U + (i + 1) * rs, n, s, un);
            rc.load(src, ld, i + 1, n);
        }
        const double vb = (bval && !a.term) ? a.V[(int64_t)b * m + i] : 0.0;
#pragma unroll
        for (int k = 0; k < kRwJ; ++k) {
            const int j = s + kRwLanes * k;
            if (FULL || j < n) w[padj(j, lg)] = cf[2 * PL + padj(j, lg)] * uc[k] + (j == 0 ? a.g_src * vb : 0.0);
        }
        wave_lds_fence();
        tridiag_solve_masked<kRwLanes, kRwSeg, FULL>(w, cf, cf + PL, a.g_wl, n, s, lg, spare);
        wave_lds_fence();
        if (bval) {
            double* out = a.node_v + ((int64_t)b * m + i) * 2 * n;
#pragma unroll
            for (int k = 0; k < kRwJ; ++k) {
                const int j = s + kRwLanes * k;
                if (FULL || j < n) __builtin_nontemporal_store(d2v{w[padj(j, lg)], uc[k]}, reinterpret_cast<d2v*>(out + 2 * j));
            }
        }
        if (i + 1 < m) rc.store(cb + ((i + 1) & 1) * 3 * PL, PL, n, lg);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRwJ; ++k) uc[k] = un[k];
    }
}

// (the unmasked solve measured 5% slower here: this walk is bound by its node-voltage
// writes, and the unmasked path holds more registers)
__global__ __launch_bounds__(256) void recover_kernel(RecoverArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    recover_walk<false>(a, smem_raw);
}

// ---------------------------------------------------------------------------
template <typename T, int NT, bool IR>
hipError_t launch_sweep_nt(const SweepArgs& a, hipStream_t s)
{
    constexpr int threads = 64 * (SweepWaves<NT>::value + SweepHelpers<IR>::value);
    const size_t lds = sweep_lds_bytes<T, NT, IR>(a.n);
    if constexpr (!IR) {
        if (a.node_v != nullptr) {
            if (a.batch > 1) return hipErrorInvalidValue;       // batches: currents only
            hipLaunchKernelGGL((sweep_kernel<T, NT, IR, true>), dim3(a.nslab), dim3(threads), lds, s, a);
            return hipGetLastError();
        }
    } else {
        if (a.batch > 1) return hipErrorInvalidValue;           // batches: float64 only
    }
    // a batch: crossbars in groups of 8 (one per XCD), a crossbar's slabs on its XCD
    const unsigned grid = a.batch > 1 ? (unsigned)(((a.batch + 7) / 8) * 8 * a.slabs_per) : (unsigned)a.nslab;
    hipLaunchKernelGGL((sweep_kernel<T, NT, IR, false>), dim3(grid), dim3(threads), lds, s, a);
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
    const size_t lds = ((size_t)xbk::kRwCols + 2 * 5) * xbk::padded_len(a.n, xbk::kRwLanes) * sizeof(double);
    hipLaunchKernelGGL(xbk::residual_kernel, dim3(2 * a.nslab), dim3(256), lds, s, a);
    return hipGetLastError();
}

hipError_t xbk_launch_recover(const xbk::RecoverArgs& a, hipStream_t s)
{
    if (a.slab_final == nullptr) return hipErrorInvalidValue;
    const size_t lds = ((size_t)xbk::kRwCols + 2 * 3) * xbk::padded_len(a.n, xbk::kRwLanes) * sizeof(double);
    hipLaunchKernelGGL(xbk::recover_kernel, dim3(2 * a.nslab), dim3(256), lds, s, a);
    return hipGetLastError();
}

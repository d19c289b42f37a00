// Pivot-block inverses of the block LU by Newton-Schulz iteration.
//
// The block LU of the condensed system (twisted order, see factor.hip) needs
// H_i = P_i^{-1} for every pivot block P_i = E_i - g_bl^2 (H_a + H_b).  The
// pivot blocks are symmetric positive definite and close to diagonal, and
// consecutive pivots of a chain differ little, so the inverse is reached in a
// few steps of the quadratically convergent Newton-Schulz iteration
//     Q_k = I - X_k P,      X_{k+1} = X_k + Q_k X_k      (I - X_{k+1} P = Q_k^2)
// started from the previous row's inverse corrected to first order in the change
// of the pivot block, with the previous inverse taken as its diagonal there,
//     X_0 = H_prev + diag(P)^{-1} - diag(P_prev)^{-1} - D offdiag(P - P_prev) D,
//     D = diag(P_prev)^{-1}
// (elementwise: for the 512 x 512 workload it takes max |I - X_0 P| from about
// 6e-6 to 5e-9 at 2.5-ohm segments and from 1.5e-5 to 2.4e-8 at 5 ohm),
// or from diag(P)^{-1} at a chain start and for the twist block.  float64 rows
// take the third-order step as a round of three launches,
//     Q = I - X P;    Y = Q X;    X'' = X + Y + Q Y = (I + Q + Q^2) X,
// whose residual is I - X'' P = Q^3: three n_p^3 products in three launches (two
// quadratic steps, with residual Q^4, cost four).  All products run on the matrix
// cores, spread over all the GPU's workgroups; no small serial inversion sits on
// the critical path.
//
// The largest |Q| entry of a round is reduced on the device (per-workgroup
// partials of the residual launch, combined by every workgroup of the round's
// last launch).  When it is <= 6.4e-5 / n_p, ||Q||_inf <= 6.4e-5 and the round
// leaves ||I - X'' P||_inf <= 2.7e-13 (in practice float64 rounding: at 512 x 512
// the warm start begins a chain's rows at about |Q| = 5e-9 to 2.4e-8, so one round
// ends at rounding level).  The float32 factor
// of the refinement mode takes single quadratic steps, stops at 1e-4 and relies on
// the refinement.  The result is
// written over E_i.  A row still above the threshold after its last round raises
// kNsFail, and the host then refactors with Gauss-Jordan elimination
// (factor.hip).
//
// The schedule is driven by the device.  The two chains are independent until
// the twist, so each runs on a stream of its own, and a third schedule inverts
// the twist block once both have finished; the launches of one chain then fill
// the matrix cores while the other's are starting up or writing out.  Each
// launch (slot) does one phase of its schedule (the form, or one launch of a
// round) and hands the next state to the following launch, so a converged row
// costs no further launches.  The launch that finishes a row also
// forms the chain's next pivot block and first iterate, element by element from
// the tile of H it has just computed, so only the chain starts and the twist
// need a form launch of their own.  The host launches the slot count the last
// factorization needed, reads the states back, and launches more until every
// schedule has finished.
//
// Every block here (E_i, H_i, S, X, Q, Y) is stored fragment-tiled (FRG), and a
// product C = A B^T is formed with the A slot of the matrix cores fed from tile
// rows of B and the B slot from tile rows of A, so that operand loads and output
// stores are all contiguous 16-byte accesses.  Since S is symmetric, X S^T = X S;
// Q X and Q Y are formed as Q X^T and Q Y^T, equal up to rounding because the
// iteration keeps X and Y symmetric (Q X = X - X P X is symmetric when X and P
// are, and so is every iterate).
#include <algorithm>

#include "common.h"

namespace xbk {

// float64: largest |Q| of a round, so that (n_p |Q|)^3 <= 2.6e-13 (see the bound above)
template <int NT>
constexpr double ns_done() { return 6.4e-5 / (64.0 * NT); }
constexpr double kNsDoneF32 = 1e-4;    // float32: at float rounding after the update

// float64 rows take third-order rounds (three launches); the float32 factor of the
// refinement mode, whose loose tolerance a warm-started row meets after one
// quadratic step, takes single steps (residual launch, update launch).
template <typename T>
constexpr bool ns_rounds() { return sizeof(T) == 8; }

template <typename T> struct V4;
template <> struct V4<double> { using type = d4_t; };
template <> struct V4<float> { using type = f4_t; };

template <typename T>
__device__ inline const T* hslot(const NSArgs& a, int row)
{
    return row < 0 ? nullptr : reinterpret_cast<const T*>(a.H) + (int64_t)row * a.n_p * a.n_p;
}

// Pivot block of row `row` in schedule `chain` (twisted order): the top chain
// takes rows 0..kt-1, the bottom chain rows m-1..kt+1, and schedule 2 the twist
// row kt = m/2 (with the top chain's buffers, once both chains have finished).
__device__ inline NSJob ns_job(int m, int chain, int row)
{
    const int kt = m / 2;
    if (chain == 2) return NSJob{kt, kt >= 1 ? kt - 1 : -1, kt + 1 <= m - 1 ? kt + 1 : -1, 0, 0};
    if (chain == 0) return NSJob{row, row > 0 ? row - 1 : -1, -1, row > 0 ? 1 : 0, 0};
    return NSJob{row, row < m - 1 ? row + 1 : -1, -1, row < m - 1 ? 1 : 0, 1};
}

// State of a schedule once `row` is inverted (xb: buffer of the next iterate).  A
// next row of the same chain starts at its first residual product: its pivot block
// and first iterate are formed by the update that finished this row.
__device__ inline NSState ns_advance(int m, int chain, int row, int slot, int xb)
{
    const int kt = m / 2;
    if (chain == 0 && row + 1 < kt) return NSState{row + 1, kNsResid, 0, xb, 0};
    if (chain == 1 && row - 1 > kt) return NSState{row - 1, kNsResid, 0, xb, 0};
    return NSState{-1, kNsFinished, 0, 0, slot + 1};
}

// Next row of a chain whose pivot block an update can form in place (-1: none).
__device__ inline int ns_fused_next(int m, int chain, int row)
{
    const int kt = m / 2;
    if (chain == 0) return row + 1 < kt ? row + 1 : -1;
    if (chain == 1) return row - 1 > kt ? row - 1 : -1;
    return -1;
}

// Form P = E_row - g^2 (H_a + H_b) and the starting iterate X_0 (identity on the
// padding); element e0, e0 + stride, ... of the FRG block.
template <typename T>
__device__ __forceinline__ void ns_form(const NSArgs& a, const NSJob& job, const NSChain& ch, int xb, int64_t e0,
                                        int64_t stride)
{
    const int n_p = a.n_p, n = a.n;
    const int64_t nn = (int64_t)n_p * n_p;
    const T* E = hslot<T>(a, job.row);
    const T* Ha = hslot<T>(a, job.dep_a);
    const T* Hb = hslot<T>(a, job.dep_b);
    T* S = reinterpret_cast<T*>(ch.S);
    T* X = reinterpret_cast<T*>(ch.X[xb]);
    double dmin = __builtin_inf();
    for (int64_t e = e0; e < nn; e += stride) {
        int r, c;
        frg_rc<T>(e, n_p, r, c);
        T s, x;
        if (r >= n || c >= n) {
            s = x = (r == c) ? (T)1 : (T)0;
        } else {
            s = E[e];
            if (Ha) s -= (T)a.g2 * Ha[e];
            if (Hb) s -= (T)a.g2 * Hb[e];
            if (job.warm) {
                x = Ha[e];
                if (r == c) x += (T)1 / s - (T)(1.0 / ch.dprev[(job.dep_a & 1) * n_p + r]);
            } else {
                x = (r == c) ? (T)1 / s : (T)0;
            }
            if (r == c) {
                ch.dprev[(job.row & 1) * n_p + r] = (double)s;
                dmin = ((double)s < dmin || s != s) ? (double)s : dmin;
            }
        }
        S[e] = s;
        X[e] = x;
    }
    record_min_pivot(dmin, a.diag, a.flags);
}

// A-operand fragment of FRG tile (tr, tk) of an n_p x n_p block (kt = n_p / 16).
template <typename T>
__device__ __forceinline__ typename V4<T>::type load_frag(const T* __restrict__ M, int kt, int tr, int tk, int l)
{
    using v4 = typename V4<T>::type;
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

// The first operand chunk of a product (this wave's first K chunk of tile rows TR,
// TR + 1 of A and TC, TC + 1 of B), when it was requested ahead (valid).
template <typename T>
struct NSFirst {
    typename V4<T>::type a[2], b[2];
    bool valid = false;
};

template <typename T, int NT>
__device__ __forceinline__ void ns_first(const T* __restrict__ Am, const T* __restrict__ Bm, int TR, int TC, int w,
                                         int l, NSFirst<T>& f)
{
    constexpr int kt = 4 * NT;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        f.a[i] = load_frag<T>(Am, kt, TR + i, w * NT, l);
        f.b[i] = load_frag<T>(Bm, kt, TC + i, w * NT, l);
    }
}

// Products of a Newton-Schulz round on a 32x32 output tile per workgroup.
// The four waves split K = n_p into quarters (NT = n_p / 64 chunks of 16
// each), every wave accumulating all four 16x16 output tiles (of one or two
// products that share the A operand); the partial sums meet in LDS and wave w
// finishes output tile w.  C = A B^T throughout, so tile row TR of A and tile
// row TC of B are read.
template <typename T, int NT, int NB>
__device__ __forceinline__ void ns_core(const T* __restrict__ Am, const T* const (&Bm)[NB], int TR, int TC, int w,
                                        int l, typename Frag<T>::acc_t (&acc)[NB][2][2], const NSFirst<T>& first)
{
    using v4 = typename V4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    constexpr int kt = 4 * NT;
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[p][i][j] = acc_t{0, 0, 0, 0};
    const int K0 = w * NT;
    v4 ac[2], bc[NB][2];
    if (ns_rounds<T>() && NB == 1 && first.valid) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ac[i] = first.a[i];
            bc[0][i] = first.b[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ac[i] = load_frag<T>(Am, kt, TR + i, K0, l);
#pragma unroll
            for (int p = 0; p < NB; ++p) bc[p][i] = load_frag<T>(Bm[p], kt, TC + i, K0, l);
        }
    }
#pragma unroll
    for (int K = 0; K < NT; ++K) {
        v4 an[2], bn[NB][2];
        if (K + 1 < NT) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                an[i] = load_frag<T>(Am, kt, TR + i, K0 + K + 1, l);
#pragma unroll
                for (int p = 0; p < NB; ++p) bn[p][i] = load_frag<T>(Bm[p], kt, TC + i, K0 + K + 1, l);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int p = 0; p < NB; ++p)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[p][i][j] = Frag<T>::mma(bc[p][j][t], ac[i][t], acc[p][i][j]);
        if (K + 1 < NT) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ac[i] = an[i];
#pragma unroll
                for (int p = 0; p < NB; ++p) bc[p][i] = bn[p][i];
            }
        }
    }
}

// Sum of the four waves' partial tiles: wave w receives output tile w.
template <typename T>
__device__ __forceinline__ typename Frag<T>::acc_t ns_reduce(const typename Frag<T>::acc_t (&acc)[2][2], T* red,
                                                              int w, int l)
{
    using acc_t = typename Frag<T>::acc_t;
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[((w * 4 + o) * 4 + v) * 64 + l] = acc[o >> 1][o & 1][v];
    __syncthreads();
    acc_t sum = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) sum[v] += red[((k * 4 + w) * 4 + v) * 64 + l];
    return sum;
}

// Largest |entry| of this workgroup's output tiles -> the chain's partial of `tile`.
template <typename T>
__device__ __forceinline__ void ns_tile_max(const NSArgs& a, int chain, int tile, int tiles, const T (&val)[4],
                                            double* wmax, int w, int l)
{
    double mx = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double av = fabs((double)val[v]);
        mx = (av > mx || av != av) ? av : mx;          // keep NaN
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(mx, off);
        mx = (o > mx || o != o) ? o : mx;
    }
    if (l == 0) wmax[w] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = wmax[0];
        for (int k = 1; k < 4; ++k) t = (wmax[k] > t || wmax[k] != wmax[k]) ? wmax[k] : t;
        a.part[(int64_t)chain * tiles + tile] = t;
    }
}

// Residual launch:  Q = I - X S and the workgroup's max |Q|.
template <typename T, int NT>
__device__ __forceinline__ void ns_resid(const NSArgs& a, const NSChain& ch, int xb, int chain, int tile, T* red,
                                         double* wmax, const NSFirst<T>& first)
{
    using acc_t = typename Frag<T>::acc_t;
    constexpr int kt = 4 * NT, tdim = 2 * NT, tiles = tdim * tdim;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4, r = l & 15;
    const int TR = 2 * (tile / tdim), TC = 2 * (tile % tdim);
    const T* const Bm[1] = {reinterpret_cast<const T*>(ch.S)};
    acc_t acc[1][2][2];
    ns_core<T, NT, 1>(reinterpret_cast<const T*>(ch.X[xb]), Bm, TR, TC, w, l, acc, first);
    const acc_t sum = ns_reduce<T>(acc[0], red, w, l);
    const int tr = TR + (w >> 1), tc = TC + (w & 1);
    T* Q = reinterpret_cast<T*>(ch.Q);
    T val[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int c = Frag<T>::kidx(q, v);
        val[v] = (T)(tr == tc && r == c ? 1 : 0) - sum[v];
        Q[((int64_t)tr * kt + tc) * 256 + frg_slot<T>(l, v)] = val[v];
    }
    ns_tile_max<T>(a, chain, tile, tiles, val, wmax, w, l);
}

// Middle launch of a round:  Y = Q X into the other iterate buffer.  It leaves the
// residual launch's max |Q| partials in place for the last launch.
template <typename T, int NT>
__device__ __forceinline__ void ns_qx(const NSArgs& a, const NSChain& ch, int xb, int tile, T* red,
                                      const NSFirst<T>& first)
{
    using acc_t = typename Frag<T>::acc_t;
    constexpr int kt = 4 * NT, tdim = 2 * NT;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int TR = 2 * (tile / tdim), TC = 2 * (tile % tdim);
    const T* X = reinterpret_cast<const T*>(ch.X[xb]);
    const int64_t base = ((int64_t)(TR + (w >> 1)) * kt + TC + (w & 1)) * 256;
    // Q X = Q X^T (X is symmetric)
    const T* const Bm[1] = {X};
    acc_t acc[1][2][2];
    ns_core<T, NT, 1>(reinterpret_cast<const T*>(ch.Q), Bm, TR, TC, w, l, acc, first);
    const acc_t qx = ns_reduce<T>(acc[0], red, w, l);
    T* Y = reinterpret_cast<T*>(ch.X[xb ^ 1]);
#pragma unroll
    for (int v = 0; v < 4; ++v) Y[base + frg_slot<T>(l, v)] = qx[v];
}

// Last launch of a round:  X'' = X + Y + Q Y with Y = Q X (Xadd = X), whose
// residual is Q^3 (or, for single steps, X' = X + Q X with residual Q^2: Y = X,
// Xadd = nullptr).  When the round converged (the largest |entry| of Q, read from
// the residual launch's partials, is <= the tolerance) or was the last allowed,
// the result is H_row; the launch
// that finishes a row also forms the chain's next pivot block E_next - g^2 H and
// first iterate H + diag(S)^-1 - diag(S_prev)^-1, element by element from its
// tile of H (E_next is read before being overwritten by H_next, many launches
// later).  Returns whether the round converged (the same answer in every
// workgroup).
template <typename T, int NT>
__device__ __forceinline__ bool ns_update(const NSArgs& a, const NSJob& job, const NSChain& ch, const T* Am,
                                          const T* Y, const T* Xadd, T* Xout, int chain, int tile, bool last,
                                          int next_row, T* red, double* wmax, const NSFirst<T>& first)
{
    using acc_t = typename Frag<T>::acc_t;
    constexpr int n_p = 64 * NT, kt = 4 * NT, tdim = 2 * NT, tiles = tdim * tdim;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int TR = 2 * (tile / tdim), TC = 2 * (tile % tdim);
    const int64_t base = ((int64_t)(TR + (w >> 1)) * kt + TC + (w & 1)) * 256;
    const int row = 16 * (TR + (w >> 1)) + (l & 15);
    // the epilogue's operands (this tile of Y and X, of the next row's E block and
    // the previous pivot diagonal) and the round's max |Q| partials are requested
    // before the product, so that their latency hides behind it
    T yin[4], xin[4], en[4], sold[4];
    double dpr = 1.0, dpc[4] = {1.0, 1.0, 1.0, 1.0};
    double mx = 0.0;
    for (int k = threadIdx.x; k < tiles; k += 256) {
        const double o = a.part[(int64_t)chain * tiles + k];
        mx = (o > mx || o != o) ? o : mx;
    }
    const T* En = reinterpret_cast<const T*>(a.H) + (int64_t)max(next_row, 0) * n_p * n_p;
    const T* Sp = reinterpret_cast<const T*>(ch.S);                    // this row's pivot block
    const double* dprev = ch.dprev + (job.row & 1) * n_p;              // and its diagonal
    const int col0 = 16 * (TC + (w & 1));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        yin[v] = Y[base + frg_slot<T>(l, v)];
        xin[v] = Xadd ? Xadd[base + frg_slot<T>(l, v)] : (T)0;
        en[v] = next_row >= 0 ? En[base + frg_slot<T>(l, v)] : (T)0;
        sold[v] = next_row >= 0 ? Sp[base + frg_slot<T>(l, v)] : (T)0;
        const int col = col0 + Frag<T>::kidx(l >> 4, v);
        if (next_row >= 0 && col < a.n) dpc[v] = dprev[col];
    }
    if (next_row >= 0 && row < a.n) dpr = dprev[row];
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(mx, off);
        mx = (o > mx || o != o) ? o : mx;
    }
    if (l == 0) wmax[w] = mx;
    const T* const Bm[1] = {Y};
    acc_t acc[1][2][2];
    ns_core<T, NT, 1>(Am, Bm, TR, TC, w, l, acc, first);
    const acc_t sum = ns_reduce<T>(acc[0], red, w, l);      // its barrier also publishes wmax
    double nu = wmax[0];
    for (int k = 1; k < 4; ++k) nu = (wmax[k] > nu || wmax[k] != wmax[k]) ? wmax[k] : nu;
    const bool fin = nu <= (sizeof(T) == 8 ? ns_done<NT>() : kNsDoneF32);   // false for NaN
    T* Hr = reinterpret_cast<T*>(a.H) + (int64_t)job.row * n_p * n_p;
    const bool form = (fin || last) && next_row >= 0;
    T* S = reinterpret_cast<T*>(ch.S);
    double dmin = __builtin_inf();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t o = base + frg_slot<T>(l, v);
        const T x = (Xadd ? xin[v] + yin[v] : yin[v]) + sum[v];
        if (fin || last) Hr[o] = x;
        if (form) {
            const int col = col0 + Frag<T>::kidx(l >> 4, v);
            T sv, xv;
            if (row >= a.n || col >= a.n) {
                sv = xv = (row == col) ? (T)1 : (T)0;
            } else {
                sv = en[v] - (T)a.g2 * x;
                xv = x;
                if (row == col) {
                    xv += (T)1 / sv - (T)(1.0 / dpr);
                    ch.dprev[(next_row & 1) * n_p + row] = (double)sv;
                    dmin = ((double)sv < dmin || sv != sv) ? (double)sv : dmin;
                } else {
                    xv -= (T)((double)(sv - sold[v]) / (dpr * dpc[v]));
                }
            }
            S[o] = sv;
            Xout[o] = xv;
        } else if (!(fin || last)) {
            Xout[o] = x;
        }
    }
    // the diagonal of the next pivot block: only waves on a diagonal tile hold it
    if (form && TR + (w >> 1) == TC + (w & 1)) record_min_pivot(dmin, a.diag, a.flags);
    return fin;
}

// One slot of schedule `chain`: its current phase, spread over (n_p/32)^2
// workgroups (a 32x32 output tile each); workgroup 0 writes the next state.  A
// finished schedule only carries its state over.
template <typename T, int NT>
__global__ __launch_bounds__(256) void ns_slot_kernel(NSArgs a, int chain, int slot)
{
    constexpr int tdim = 2 * NT;
    __shared__ __align__(16) T red[4 * 4 * 4 * 64];       // product partials [wave][output tile][item][lane]
    __shared__ double wmax[4];
    // XCD-aware tile map: workgroups are dispatched round-robin over the 8 XCDs
    // (each with its own L2), so workgroup b runs on XCD b % 8.  Each XCD owns a
    // block of a quarter of the tile rows and half of the tile columns, so its L2
    // holds a quarter of the rows of one operand and half of the other's.
    int tile = blockIdx.x;
    if constexpr (tdim % 4 == 0) {
        constexpr int rpx = tdim / 4, cpx = tdim / 2;
        const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
        tile = ((xcd >> 1) * rpx + local / cpx) * tdim + (xcd & 1) * cpx + local % cpx;
    }
    const NSState* cur = a.state + 3 * (slot & 1);
    NSState* nxt = a.state + 3 * ((slot + 1) & 1);
    const int m = a.m;
    // float64 rounds keep the iterate in X[0], and a schedule's launches take its
    // phases in a fixed order (a form, then residual, Q X and update launches in
    // turn) until it finishes.  So this slot's first operand chunk is requested
    // before its state has arrived; a state that disagrees (a finished schedule)
    // leaves it unused.  (The float32 steps' short launches measured slower with it.)
    NSFirst<T> first;
    int guess = -1;
    if constexpr (ns_rounds<T>()) {
        if (slot > 0) {
            guess = kNsResid + (slot - 1) % 3;
            const NSChain& cg = a.ch[chain == 1 ? 1 : 0];
            const T* Ag = reinterpret_cast<const T*>(guess == kNsResid ? cg.X[0] : cg.Q);
            const T* Bg = reinterpret_cast<const T*>(guess == kNsResid ? cg.S : cg.X[guess == kNsQx ? 0 : 1]);
            ns_first<T, NT>(Ag, Bg, 2 * (tile / tdim), 2 * (tile % tdim), threadIdx.x >> 6, threadIdx.x & 63, first);
        }
    }
    const NSState s = cur[chain];
    first.valid = s.phase == guess && s.xb == 0;
    NSState ns = s;
    if (s.phase != kNsFinished) {
        const NSJob job = ns_job(m, chain, s.row);
        const NSChain& ch = a.ch[job.chain];
        if (s.phase == kNsForm) {
            constexpr int tiles = tdim * tdim;
            ns_form<T>(a, job, ch, s.xb, (int64_t)tile * 256 + threadIdx.x, (int64_t)tiles * 256);
            ns = NSState{s.row, kNsResid, 0, s.xb, 0};
        } else if (s.phase == kNsResid) {
            ns_resid<T, NT>(a, ch, s.xb, job.chain, tile, red, wmax, first);
            ns = NSState{s.row, ns_rounds<T>() ? kNsQx : kNsUpdate, s.it, s.xb, 0};
        } else if (s.phase == kNsQx) {
            ns_qx<T, NT>(a, ch, s.xb, tile, red, first);
            ns = NSState{s.row, kNsUpdate, s.it, s.xb, 0};
        } else {
            // a round: X[xb] <- X + Y + Q Y with Y = Q X in X[xb^1] (in place: each
            // workgroup reads only its own tile of X); a single step: X[xb^1] <- X + Q X
            constexpr int steps = ns_rounds<T>() ? 2 : 1;
            T* const X0 = reinterpret_cast<T*>(ch.X[s.xb]);
            T* const X1 = reinterpret_cast<T*>(ch.X[s.xb ^ 1]);
            const T* Am = reinterpret_cast<const T*>(ch.Q);
            const int xo = ns_rounds<T>() ? s.xb : s.xb ^ 1;
            const int maxit = job.warm ? a.max_iter : a.max_iter + 4;
            const bool last = s.it + steps >= maxit;
            const int next_row = ns_fused_next(m, chain, s.row);
            const bool fin = ns_update<T, NT>(a, job, ch, Am, ns_rounds<T>() ? X1 : X0, ns_rounds<T>() ? X0 : nullptr,
                                              ns_rounds<T>() ? X0 : X1, job.chain, tile, last, next_row, red, wmax,
                                              first);
            if (fin || last) {
                if (!fin && tile == 0 && threadIdx.x == 0) atomicOr(a.flags + kNsFail, 1);
                ns = ns_advance(m, chain, s.row, slot, xo);
            } else {
                ns = NSState{s.row, kNsResid, s.it + steps, xo, 0};
            }
        }
    }
    if (tile == 0 && threadIdx.x == 0) nxt[chain] = ns;
}

__global__ void ns_init_kernel(NSArgs a)
{
    if (threadIdx.x != 0) return;
    const int m = a.m, kt = m / 2;
    a.state[0] = kt > 0 ? NSState{0, kNsForm, 0, 0, 0} : NSState{-1, kNsFinished, 0, 0, 0};
    a.state[1] = m - 1 > kt ? NSState{m - 1, kNsForm, 0, 0, 0} : NSState{-1, kNsFinished, 0, 0, 0};
    a.state[2] = NSState{kt, kNsForm, 0, 0, 0};
}

// After the schedules' launch budgets: the launches each schedule needed
// (kNsUsed + c, 0 for one that had not finished), and kErrConv when a row missed
// its tolerance (kNsFail) or a schedule had not finished within its budget.
__global__ void ns_finish_kernel(NSArgs a, int l0, int l1, int l2)
{
    if (threadIdx.x != 0) return;
    const int launched[3] = {l0, l1, l2};
    bool open = false;
    for (int c = 0; c < 3; ++c) {
        const NSState s = a.state[3 * (launched[c] & 1) + c];
        const bool fin = s.phase == kNsFinished;
        open |= !fin;
        a.flags[kNsUsed + c] = fin ? s.slots : 0;
    }
    if (open || a.flags[kNsFail]) a.flags[kErrConv] = 1;
}

template <typename T, int NT>
hipError_t launch_slots_nt(const NSArgs& a, int chain, int first, int count, hipStream_t s)
{
    constexpr int tiles = (2 * NT) * (2 * NT);
    for (int k = 0; k < count; ++k) {
        hipLaunchKernelGGL((ns_slot_kernel<T, NT>), dim3(tiles), dim3(256), 0, s, a, chain, first + k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_slots(const NSArgs& a, int chain, int first, int count, hipStream_t s)
{
    switch (a.n_p / 64) {
        case 1: return launch_slots_nt<T, 1>(a, chain, first, count, s);
        case 2: return launch_slots_nt<T, 2>(a, chain, first, count, s);
        case 3: return launch_slots_nt<T, 3>(a, chain, first, count, s);
        case 4: return launch_slots_nt<T, 4>(a, chain, first, count, s);
        case 5: return launch_slots_nt<T, 5>(a, chain, first, count, s);
        case 6: return launch_slots_nt<T, 6>(a, chain, first, count, s);
        case 7: return launch_slots_nt<T, 7>(a, chain, first, count, s);
        case 8: return launch_slots_nt<T, 8>(a, chain, first, count, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace xbk

hipError_t xbk_launch_ns_init(const xbk::NSArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::ns_init_kernel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t xbk_launch_ns_slots(const xbk::NSArgs& a, bool fp32, int chain, int first, int count, hipStream_t s)
{
    if (chain < 0 || chain > 2) return hipErrorInvalidValue;
    return fp32 ? xbk::launch_slots<float>(a, chain, first, count, s)
                : xbk::launch_slots<double>(a, chain, first, count, s);
}

hipError_t xbk_launch_ns_finish(const xbk::NSArgs& a, int launched0, int launched1, int launched2, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::ns_finish_kernel, dim3(1), dim3(64), 0, s, a, launched0, launched1, launched2);
    return hipGetLastError();
}

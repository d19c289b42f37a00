// Pivot-block inverses of the block LU by Newton-Schulz iteration.
//
// The block LU of the condensed system (twisted order, see factor.hip) needs
// H_i = P_i^{-1} for every pivot block P_i = E_i - g_bl^2 (H_a + H_b).  The
// pivot blocks are symmetric positive definite and close to diagonal, and
// consecutive pivots of a chain differ little, so the inverse is reached in a
// few steps of the quadratically convergent iteration
//     Q_k = I - X_k P,      X_{k+1} = X_k + Q_k X_k      (I - X_{k+1} P = Q_k^2)
// started from the previous row's inverse with its diagonal corrected,
//     X_0 = H_prev + diag(P)^{-1} - diag(P_prev)^{-1},
// or from diag(P)^{-1} at a chain start and for the twist block.  Every step
// is two n_p^3 products on the matrix cores, spread over all the GPU's
// workgroups; no small serial inversion sits on the critical path.
//
// The largest |Q_k| entry is reduced on the device (per-workgroup partials,
// combined by every workgroup of the following update).  When it is <= 1e-9,
// ||Q_k||_inf <= n_p 1e-9 and the update just applied leaves
// ||I - X_{k+1} P||_inf <= (n_p 1e-9)^2 <= 2.7e-13 for n_p <= 512 (in practice
// float64 rounding: consecutive pivots of a chain start the iteration at about
// 4e-6, then 3e-10, then 3e-15).  The float32 factor of the refinement mode
// stops at 1e-4 and relies on the refinement.  The result is written over E_i
// and later launches for the row exit at once.  A row still
// above the threshold after its last step raises kNsFail, and the host then
// refactors with Gauss-Jordan elimination (factor.hip).
//
// The schedule is driven by the device: each launch (slot) does one phase per
// chain (form, residual product, update product) and hands the chain's next
// state to the following launch, so a converged row costs no further launches.
// The update that finishes a row also forms the chain's next pivot block and
// first iterate, element by element from the tile of H it has just computed, so
// only the chain starts and the twist need a form launch of their own.
// The host launches an estimate of the slots needed, reads the two states
// back, and launches more until both chains have finished.
//
// Every block here (E_i, H_i, S, X, Q) is stored fragment-tiled (FRG), and
// a product C = A B^T is formed with the A slot of the matrix cores fed from
// tile rows of B and the B slot from tile rows of A, so that operand loads and
// output stores are all contiguous 16-byte accesses.  Since S is symmetric,
// X S^T = X S; the update uses Q X^T, which equals Q X up to rounding because
// the iteration keeps X symmetric (2X - X S X is symmetric when X is).
#include <algorithm>

#include "common.h"

namespace xbk {

constexpr double kNsDone = 1e-9;       // float64: see the bound above
constexpr double kNsDoneF32 = 1e-4;    // float32: at float rounding after the update

template <typename T> struct V4;
template <> struct V4<double> { using type = d4_t; };
template <> struct V4<float> { using type = f4_t; };

template <typename T>
__device__ inline const T* hslot(const NSArgs& a, int row)
{
    return row < 0 ? nullptr : reinterpret_cast<const T*>(a.H) + (int64_t)row * a.n_p * a.n_p;
}

// Pivot block of row `row` in chain `chain` (twisted order): the top chain takes rows
// 0..kt-1 and then the twist row kt = m/2, the bottom chain rows m-1..kt+1.
__device__ inline NSJob ns_job(int m, int chain, int row)
{
    const int kt = m / 2;
    if (row == kt) return NSJob{kt, kt >= 1 ? kt - 1 : -1, kt + 1 <= m - 1 ? kt + 1 : -1, 0, 0};
    if (chain == 0) return NSJob{row, row > 0 ? row - 1 : -1, -1, row > 0 ? 1 : 0, 0};
    return NSJob{row, row < m - 1 ? row + 1 : -1, -1, row < m - 1 ? 1 : 0, 1};
}

// State of a chain once `row` is inverted (xb: buffer of the next iterate).  A next
// row of the same chain starts at its first residual product: its pivot block and
// first iterate are formed by the update that finished this row.
__device__ inline NSState ns_advance(int m, int chain, int row, int slot, int xb)
{
    const int kt = m / 2;
    if (chain == 0) {
        if (row == kt) return NSState{row, kNsFinished, 0, 0, slot + 1};
        if (row + 1 < kt) return NSState{row + 1, kNsResid, 0, xb, 0};
        return NSState{kt, kNsWait, 0, 0, 0};        // the twist needs the bottom chain's last inverse
    }
    if (row - 1 > kt) return NSState{row - 1, kNsResid, 0, xb, 0};
    return NSState{-1, kNsFinished, 0, 0, slot + 1};
}

// Next row of a chain whose pivot block an update can form in place (-1: none).
__device__ inline int ns_fused_next(int m, int chain, int row)
{
    const int kt = m / 2;
    if (row == kt) return -1;
    if (chain == 0) return row + 1 < kt ? row + 1 : -1;
    return row - 1 > kt ? row - 1 : -1;
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
                if (r == c) x += (T)1 / s - (T)(1.0 / ch.dprev[r]);
            } else {
                x = (r == c) ? (T)1 / s : (T)0;
            }
            if (r == c) ch.dprev[r] = (double)s;
        }
        S[e] = s;
        X[e] = x;
    }
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

// One product of a Newton-Schulz step on a 32x32 output tile per workgroup.
// The four waves split K = n_p into quarters (NT = n_p / 64 chunks of 16
// each), every wave accumulating all four 16x16 output tiles; the partial
// sums meet in LDS and wave w finishes output tile w.
//   MODE 0:  Q = I - X_k S          (and the workgroup's max |Q|)
//   MODE 1:  X_{k+1} = X_k + Q X_k  (and H_row when the step converged or was the last)
// MODE 1 returns whether the step converged (the same answer in every workgroup).
template <typename T, int MODE, int NT>
__device__ __forceinline__ bool ns_product(const NSArgs& a, const NSJob& job, const NSChain& ch, int xb,
                                           int chain, int tile, bool last, int next_row, T* red, double* wmax)
{
    using v4 = typename V4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    constexpr int n_p = 64 * NT, kt = n_p / 16, tdim = n_p / 32, tiles = tdim * tdim;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int TR = 2 * (tile / tdim), TC = 2 * (tile % tdim);
    const T* Xin = reinterpret_cast<const T*>(ch.X[xb]);
    // C = Am Bm^T
    const T* Am = MODE == 0 ? Xin : reinterpret_cast<const T*>(ch.Q);
    const T* Bm = MODE == 0 ? reinterpret_cast<const T*>(ch.S) : Xin;
    acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    const int K0 = w * NT;
    v4 ac[2], bc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        ac[i] = load_frag<T>(Am, kt, TR + i, K0, l);
        bc[i] = load_frag<T>(Bm, kt, TC + i, K0, l);
    }
#pragma unroll
    for (int K = 0; K < NT; ++K) {
        v4 an[2], bn[2];
        if (K + 1 < NT) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                an[i] = load_frag<T>(Am, kt, TR + i, K0 + K + 1, l);
                bn[i] = load_frag<T>(Bm, kt, TC + i, K0 + K + 1, l);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Frag<T>::mma(bc[j][t], ac[i][t], acc[i][j]);
        if (K + 1 < NT) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ac[i] = an[i];
                bc[i] = bn[i];
            }
        }
    }
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
    // wave w owns output tile (TR + w/2, TC + w%2); lane l item v is (row, col) of C
    const int64_t base = ((int64_t)(TR + (w >> 1)) * kt + TC + (w & 1)) * 256;
    const int row = 16 * (TR + (w >> 1)) + (l & 15);
    double* part = a.part + (int64_t)chain * tiles;    // this chain's partials
    if (MODE == 0) {
        T* Q = reinterpret_cast<T*>(ch.Q);
        double mx = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = 16 * (TC + (w & 1)) + Frag<T>::kidx(l >> 4, v);
            const T val = (T)(row == col ? 1 : 0) - sum[v];
            Q[base + frg_slot<T>(l, v)] = val;
            const double av = fabs((double)val);
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
            part[tile] = t;
        }
        return false;
    } else {
        // max over the chain's workgroup partials of Q's step
        double mx = 0.0;
        for (int k = threadIdx.x; k < tiles; k += 256) {
            const double o = part[k];
            mx = (o > mx || o != o) ? o : mx;
        }
        wmax[threadIdx.x] = mx;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                const double o = wmax[threadIdx.x + h];
                wmax[threadIdx.x] = (o > wmax[threadIdx.x] || o != o) ? o : wmax[threadIdx.x];
            }
            __syncthreads();
        }
        const double nu = wmax[0];
        const bool fin = nu <= (sizeof(T) == 8 ? kNsDone : kNsDoneF32);   // false for NaN
        T* Xout = reinterpret_cast<T*>(ch.X[xb ^ 1]);
        T* Hr = reinterpret_cast<T*>(a.H) + (int64_t)job.row * n_p * n_p;
        const bool form = (fin || last) && next_row >= 0;
        // the next row's pivot block E_next - g^2 H and first iterate H + diag(S)^-1 - diag(S_prev)^-1,
        // element by element from this tile of H (E_next is read before being overwritten
        // by H_next, many launches later)
        const T* En = reinterpret_cast<const T*>(a.H) + (int64_t)max(next_row, 0) * n_p * n_p;
        T* S = reinterpret_cast<T*>(ch.S);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t o = base + frg_slot<T>(l, v);
            const T x = Xin[o] + sum[v];
            if (fin || last) Hr[o] = x;
            if (form) {
                const int col = 16 * (TC + (w & 1)) + Frag<T>::kidx(l >> 4, v);
                T sv, xv;
                if (row >= a.n || col >= a.n) {
                    sv = xv = (row == col) ? (T)1 : (T)0;
                } else {
                    sv = En[o] - (T)a.g2 * x;
                    xv = x;
                    if (row == col) {
                        xv += (T)1 / sv - (T)(1.0 / ch.dprev[row]);
                        ch.dprev[row] = (double)sv;
                    }
                }
                S[o] = sv;
                Xout[o] = xv;
            } else {
                Xout[o] = x;
            }
        }
        return fin;
    }
}

// One slot of the schedule: every chain does its current phase with its share of
// the grid ((n_p/32)^2 workgroups per chain), and workgroup 0 of the chain writes
// the chain's next state.  A chain that waits or has finished only carries its
// state over.
template <typename T, int NT>
__global__ __launch_bounds__(256) void ns_slot_kernel(NSArgs a, int slot)
{
    constexpr int tdim = 2 * NT, tiles = tdim * tdim, half = tdim / 2;
    __shared__ __align__(16) T red[4 * 4 * 4 * 64];       // product partials [wave][output tile][item][lane]
    __shared__ double wmax[256];
    // XCD-aware tile map: workgroups are dispatched round-robin over the 8 XCDs
    // (each with its own L2), so workgroup b runs on XCD b % 8.  XCDs 0-3 take the
    // top chain and 4-7 the bottom one; within a chain each XCD owns a quadrant of
    // the output tile grid, so its L2 holds half the rows of each operand instead
    // of all of them.
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    const int chain = xcd >> 2, quad = xcd & 3;
    const int tile = ((quad >> 1) * half + local / half) * tdim + (quad & 1) * half + local % half;
    const NSState* cur = a.state + 2 * (slot & 1);
    NSState* nxt = a.state + 2 * ((slot + 1) & 1);
    const int m = a.m;
    NSState s = cur[chain];
    if (s.phase == kNsWait && cur[1].phase == kNsFinished) s = NSState{m / 2, kNsForm, 0, 0, 0};
    NSState ns = s;
    if (s.phase == kNsForm || s.phase == kNsResid || s.phase == kNsUpdate) {
        const NSJob job = ns_job(m, chain, s.row);
        const NSChain& ch = a.ch[job.chain];
        const int maxit = job.warm ? a.max_iter : a.max_iter + 4;
        if (s.phase == kNsForm) {
            ns_form<T>(a, job, ch, s.xb, (int64_t)tile * 256 + threadIdx.x, (int64_t)tiles * 256);
            ns = NSState{s.row, kNsResid, 0, s.xb, 0};
        } else if (s.phase == kNsResid) {
            ns_product<T, 0, NT>(a, job, ch, s.xb, chain, tile, false, -1, red, wmax);
            ns = NSState{s.row, kNsUpdate, s.it, s.xb, 0};
        } else {
            const bool last = s.it + 1 >= maxit;
            const int next_row = ns_fused_next(m, chain, s.row);
            const bool fin = ns_product<T, 1, NT>(a, job, ch, s.xb, chain, tile, last, next_row, red, wmax);
            if (fin || last) {
                if (!fin && tile == 0 && threadIdx.x == 0) atomicOr(a.flags + kNsFail, 1);
                ns = ns_advance(m, chain, s.row, slot, s.xb ^ 1);
            } else {
                ns = NSState{s.row, kNsResid, s.it + 1, s.xb ^ 1, 0};
            }
        }
    }
    if (tile == 0 && threadIdx.x == 0) nxt[chain] = ns;
}

__global__ void ns_init_kernel(NSArgs a)
{
    if (threadIdx.x != 0) return;
    const int m = a.m, kt = m / 2;
    a.state[0] = kt > 0 ? NSState{0, kNsForm, 0, 0, 0} : NSState{kt, kNsWait, 0, 0, 0};
    a.state[1] = m - 1 > kt ? NSState{m - 1, kNsForm, 0, 0, 0} : NSState{-1, kNsFinished, 0, 0, 0};
}

template <typename T, int NT>
hipError_t launch_slots_nt(const NSArgs& a, int first, int count, hipStream_t s)
{
    constexpr int tiles = (2 * NT) * (2 * NT);
    for (int k = 0; k < count; ++k) {
        hipLaunchKernelGGL((ns_slot_kernel<T, NT>), dim3(2 * tiles), dim3(256), 0, s, a, first + k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_slots(const NSArgs& a, int first, int count, hipStream_t s)
{
    switch (a.n_p / 64) {
        case 1: return launch_slots_nt<T, 1>(a, first, count, s);
        case 2: return launch_slots_nt<T, 2>(a, first, count, s);
        case 3: return launch_slots_nt<T, 3>(a, first, count, s);
        case 4: return launch_slots_nt<T, 4>(a, first, count, s);
        case 5: return launch_slots_nt<T, 5>(a, first, count, s);
        case 6: return launch_slots_nt<T, 6>(a, first, count, s);
        case 7: return launch_slots_nt<T, 7>(a, first, count, s);
        case 8: return launch_slots_nt<T, 8>(a, first, count, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace xbk

hipError_t xbk_launch_ns_init(const xbk::NSArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(xbk::ns_init_kernel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t xbk_launch_ns_slots(const xbk::NSArgs& a, bool fp32, int first, int count, hipStream_t s)
{
    return fp32 ? xbk::launch_slots<float>(a, first, count, s) : xbk::launch_slots<double>(a, first, count, s);
}

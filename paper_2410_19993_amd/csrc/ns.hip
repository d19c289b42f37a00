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
// combined by every workgroup of the following update).  When it is <= 1e-10 the
// update just applied leaves an error <= 1e-20 (plus rounding; 1e-4 and 1e-8
// for the float32 factor of the refinement mode), the result is
// written over E_i and later launches for the row exit at once.  A row still
// above the threshold after its last step raises kNsFail, and the host then
// refactors with Gauss-Jordan elimination (factor.hip).
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

constexpr double kNsDone = 1e-10;      // float64: update leaves <= 1e-20 + rounding
constexpr double kNsDoneF32 = 1e-4;    // float32: update leaves <= 1e-8, at float rounding

template <typename T> struct V4;
template <> struct V4<double> { using type = d4_t; };
template <> struct V4<float> { using type = f4_t; };

template <typename T>
__device__ inline const T* hslot(const NSArgs& a, int row)
{
    return row < 0 ? nullptr : reinterpret_cast<const T*>(a.H) + (int64_t)row * a.n_p * a.n_p;
}

// Form P = E_row - g^2 (H_a + H_b) and the starting iterate X_0 (identity on the padding).
template <typename T>
__global__ __launch_bounds__(256) void ns_form_kernel(NSArgs a)
{
    const int n_p = a.n_p, n = a.n;
    const int64_t nn = (int64_t)n_p * n_p;
    const NSJob& job = a.job[blockIdx.y];
    const NSChain& ch = a.ch[job.chain];
    const T* E = hslot<T>(a, job.row);
    const T* Ha = hslot<T>(a, job.dep_a);
    const T* Hb = hslot<T>(a, job.dep_b);
    T* S = reinterpret_cast<T*>(ch.S);
    T* X = reinterpret_cast<T*>(ch.X[0]);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.done[job.row] = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
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
//   MODE 0:  Q = I - X_k S          (and the row's max |Q|)
//   MODE 1:  X_{k+1} = X_k + Q X_k  (and H_row when the step converged)
template <typename T, int MODE, int NT>
__global__ __launch_bounds__(256) void ns_gemm_kernel(NSArgs a, int it)
{
    using v4 = typename V4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    constexpr int n_p = 64 * NT, kt = n_p / 16, tdim = n_p / 32, tiles = tdim * tdim;
    __shared__ __align__(16) T red[4 * 4 * 4 * 64];       // [wave][output tile][item][lane]
    __shared__ double wmax[256];
    const NSJob& job = a.job[blockIdx.x / tiles];
    if (a.done[job.row]) return;
    const int maxit = job.warm ? a.max_iter : a.max_iter + 4;
    if (it >= maxit) return;
    const NSChain& ch = a.ch[job.chain];
    const int tile = blockIdx.x % tiles;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int TR = 2 * (tile / tdim), TC = 2 * (tile % tdim);
    const T* Xin = reinterpret_cast<const T*>(ch.X[it & 1]);
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
    double* part = a.part + (int64_t)(blockIdx.x / tiles) * tiles;    // this job's partials
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
    } else {
        // max over the job's workgroup partials of Q's step
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
        T* Xout = reinterpret_cast<T*>(ch.X[(it + 1) & 1]);
        T* Hr = reinterpret_cast<T*>(a.H) + (int64_t)job.row * n_p * n_p;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t o = base + frg_slot<T>(l, v);
            const T x = Xin[o] + sum[v];
            Xout[o] = x;
            if (fin) Hr[o] = x;
        }
        if (fin) {
            if (threadIdx.x == 0) a.done[job.row] = 1;
        } else if (it == maxit - 1 && threadIdx.x == 0 && tile == 0) {
            atomicOr(a.flags + kNsFail, 1);
        }
    }
}

template <typename T, int MODE, int NT>
hipError_t launch_gemm_nt(const NSArgs& f, int njobs, int it, hipStream_t s)
{
    constexpr int tiles = (2 * NT) * (2 * NT);
    hipLaunchKernelGGL((ns_gemm_kernel<T, MODE, NT>), dim3(njobs * tiles), dim3(256), 0, s, f, it);
    return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_gemm(const NSArgs& f, int njobs, int it, hipStream_t s)
{
    switch (f.n_p / 64) {
        case 1: return launch_gemm_nt<T, MODE, 1>(f, njobs, it, s);
        case 2: return launch_gemm_nt<T, MODE, 2>(f, njobs, it, s);
        case 3: return launch_gemm_nt<T, MODE, 3>(f, njobs, it, s);
        case 4: return launch_gemm_nt<T, MODE, 4>(f, njobs, it, s);
        case 5: return launch_gemm_nt<T, MODE, 5>(f, njobs, it, s);
        case 6: return launch_gemm_nt<T, MODE, 6>(f, njobs, it, s);
        case 7: return launch_gemm_nt<T, MODE, 7>(f, njobs, it, s);
        case 8: return launch_gemm_nt<T, MODE, 8>(f, njobs, it, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_ns(NSArgs a, hipStream_t s)
{
    const int m = a.m, kt = m / 2, n_p = a.n_p;
    const int top_len = kt, bot_len = m - 1 - kt;
    const int form_blocks = (int)std::min<int64_t>(((int64_t)n_p * n_p + 255) / 256, 1024);
    hipError_t e;
    auto run = [&](const NSArgs& f, int njobs, int iters) -> hipError_t {
        hipLaunchKernelGGL(ns_form_kernel<T>, dim3(form_blocks, njobs), dim3(256), 0, s, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int it = 0; it < iters; ++it) {
            if ((e = launch_gemm<T, 0>(f, njobs, it, s)) != hipSuccess) return e;
            if ((e = launch_gemm<T, 1>(f, njobs, it, s)) != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const int steps = top_len > bot_len ? top_len : bot_len;
    for (int st = 0; st < steps; ++st) {
        NSArgs f = a;
        int nj = 0;
        if (st < top_len) {
            f.job[nj] = NSJob{st, st > 0 ? st - 1 : -1, -1, st > 0 ? 1 : 0, 0};
            ++nj;
        }
        if (st < bot_len) {
            const int row = m - 1 - st;
            f.job[nj] = NSJob{row, st > 0 ? row + 1 : -1, -1, st > 0 ? 1 : 0, 1};
            ++nj;
        }
        if ((e = run(f, nj, st > 0 ? a.max_iter : a.max_iter + 4)) != hipSuccess) return e;
    }
    NSArgs f = a;
    f.job[0] = NSJob{kt, kt >= 1 ? kt - 1 : -1, kt + 1 <= m - 1 ? kt + 1 : -1, 0, 0};
    return run(f, 1, a.max_iter + 4);
}

}  // namespace xbk

hipError_t xbk_launch_factor_ns(const xbk::NSArgs& a, bool fp32, hipStream_t s)
{
    return fp32 ? xbk::launch_ns<float>(a, s) : xbk::launch_ns<double>(a, s);
}

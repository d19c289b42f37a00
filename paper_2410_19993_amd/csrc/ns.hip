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
// Products read both operands row-wise: the right operand (P or X) is
// symmetric, so its column k is its row k.
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
        const int r = (int)(e / n_p), p = (int)(e % n_p);
        const int c = (p & ~15) + Frag<T>::slot(p & 15);         // CPR position p holds column c
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

// One product of a Newton-Schulz step on a 32x32 output tile per workgroup
// (four waves, one 16x16 MFMA tile each, K = n_p).
//   MODE 0:  Q = I - X_k P       (and the row's max |Q|)
//   MODE 1:  X_{k+1} = X_k + Q X_k   (and H_row when the step converged)
template <typename T, int MODE>
__global__ __launch_bounds__(256) void ns_gemm_kernel(NSArgs a, int it)
{
    using v4 = typename V4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    const int n_p = a.n_p, tdim = n_p / 32, tiles = tdim * tdim;
    const NSJob& job = a.job[blockIdx.x / tiles];
    if (a.done[job.row]) return;
    const int maxit = job.warm ? a.max_iter : a.max_iter + 4;
    if (it >= maxit) return;
    const NSChain& ch = a.ch[job.chain];
    const int tile = blockIdx.x % tiles;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4, r = l & 15;
    const int R0 = 32 * (tile / tdim) + 16 * (w >> 1), C0 = 32 * (tile % tdim) + 16 * (w & 1);
    const T* Xin = reinterpret_cast<const T*>(ch.X[it & 1]);
    const T* A = MODE == 0 ? Xin : reinterpret_cast<const T*>(ch.Q);
    const T* Bm = MODE == 0 ? reinterpret_cast<const T*>(ch.S) : Xin;
    const T* ap = A + (int64_t)(R0 + r) * n_p + 4 * q;
    const T* bp = Bm + (int64_t)(C0 + r) * n_p + 4 * q;
    acc_t acc = acc_t{0, 0, 0, 0};
    // K in chunks of 16, four chunks in flight ahead of the matrix cores
    constexpr int D = 4;
    const int KC = n_p / 16;                 // a multiple of 4 (n_p is a multiple of 64)
    v4 ac[D], bc[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        ac[j] = *reinterpret_cast<const v4*>(ap + 16 * j);
        bc[j] = *reinterpret_cast<const v4*>(bp + 16 * j);
    }
    for (int K = 0; K < KC; K += D) {
        v4 an[D], bn[D];
        const bool more = K + D < KC;
        if (more) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                an[j] = *reinterpret_cast<const v4*>(ap + 16 * (K + D + j));
                bn[j] = *reinterpret_cast<const v4*>(bp + 16 * (K + D + j));
            }
        }
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = Frag<T>::mma(ac[j][t], bc[j][t], acc);
        if (more) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                ac[j] = an[j];
                bc[j] = bn[j];
            }
        }
    }
    double* part = a.part + (int64_t)(blockIdx.x / tiles) * tiles;    // this job's partials
    if (MODE == 0) {
        T* Q = reinterpret_cast<T*>(ch.Q);
        double mx = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = R0 + Frag<T>::drow(q, v), col = C0 + r;
            const T val = (T)(row == col ? 1 : 0) - acc[v];
            Q[cpr<T>(row, col, n_p)] = val;
            const double av = fabs((double)val);
            mx = (av > mx || av != av) ? av : mx;          // keep NaN
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(mx, off);
            mx = (o > mx || o != o) ? o : mx;
        }
        __shared__ double wmax[4];
        if (l == 0) wmax[w] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = wmax[0];
            for (int k = 1; k < 4; ++k) t = (wmax[k] > t || wmax[k] != wmax[k]) ? wmax[k] : t;
            part[tile] = t;
        }
    } else {
        // max over the job's workgroup partials of Q's step
        __shared__ double red[256];
        double mx = 0.0;
        for (int k = threadIdx.x; k < tiles; k += 256) {
            const double o = part[k];
            mx = (o > mx || o != o) ? o : mx;
        }
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                const double o = red[threadIdx.x + h];
                red[threadIdx.x] = (o > red[threadIdx.x] || o != o) ? o : red[threadIdx.x];
            }
            __syncthreads();
        }
        const double nu = red[0];
        const bool fin = nu <= (sizeof(T) == 8 ? kNsDone : kNsDoneF32);   // false for NaN
        T* Xout = reinterpret_cast<T*>(ch.X[(it + 1) & 1]);
        T* Hr = reinterpret_cast<T*>(a.H) + (int64_t)job.row * n_p * n_p;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t o = cpr<T>(R0 + Frag<T>::drow(q, v), C0 + r, n_p);
            const T x = Xin[o] + acc[v];
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

template <typename T>
hipError_t launch_ns(NSArgs a, hipStream_t s)
{
    const int m = a.m, kt = m / 2, n_p = a.n_p;
    const int tiles = (n_p / 32) * (n_p / 32);
    const int top_len = kt, bot_len = m - 1 - kt;
    const int form_blocks = (int)std::min<int64_t>(((int64_t)n_p * n_p + 255) / 256, 1024);
    hipError_t e;
    auto run = [&](const NSArgs& f, int njobs, int iters) -> hipError_t {
        hipLaunchKernelGGL(ns_form_kernel<T>, dim3(form_blocks, njobs), dim3(256), 0, s, f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int it = 0; it < iters; ++it) {
            hipLaunchKernelGGL((ns_gemm_kernel<T, 0>), dim3(njobs * tiles), dim3(256), 0, s, f, it);
            hipLaunchKernelGGL((ns_gemm_kernel<T, 1>), dim3(njobs * tiles), dim3(256), 0, s, f, it);
            if ((e = hipGetLastError()) != hipSuccess) return e;
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

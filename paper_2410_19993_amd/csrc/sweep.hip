// Forward and back substitution over the row blocks (Sec. II.C: L y = I then
// U v = y, for every input vector of a batch, Sec. III.A/III.D), in the
// twisted order of the factorization (top chain rows 0..kt-1, bottom chain
// rows m-1..kt+1, twist row kt = m/2), with H_i the stored pivot inverses:
//   forward, top:    y_0 = f_0,        z_i = H_i y_i,  y_{i+1} = f_{i+1} + g_bl z_i
//   forward, bottom: y_{m-1} = f_{m-1}, z_i = H_i y_i,  y_{i-1} = f_{i-1} + g_bl z_i
//   twist:           u_kt = H_kt (f_kt + g_bl z_{kt-1} + g_bl z_{kt+1})
//   back, up:        u_i = z_i + g_bl H_i u_{i+1}   (i = kt-1 .. 0)
//   back, down:      u_i = z_i + g_bl H_i u_{i-1}   (i = kt+1 .. m-1)
// with f_i = V_i c_i.  Output currents are I_j = g_sense u_{m-1, j}.
//
// Input vectors are independent, so each workgroup owns a slab of 16 of
// them for the whole sweep: no grid synchronisation at all.  Per row block
// it computes an (n_p x n_p) x (n_p x 16) product on the matrix cores: H_i
// streams from L2/HBM straight into registers as MFMA A fragments, and the
// 16-column right-hand-side panel sits in LDS.  Wave w owns output rows
// [w n_p/4, (w+1) n_p/4), NT = n_p/64 tiles of 16 rows.
#include "common.h"

namespace xbk {

template <typename T> struct Vec4;
template <> struct Vec4<double> { using type = d4_t; };
template <> struct Vec4<float> { using type = f4_t; };

// k position inside a CPR row (16-chunk permuted)
template <typename T>
__device__ __host__ inline int pos(int k) { return (k & ~15) + Frag<T>::slot(k & 15); }

template <typename T, int NT>
__device__ inline void panel_product(typename Frag<T>::acc_t (&acc)[NT], const T* __restrict__ Hi,
                                     const T* ybuf, int ldy, int w, int l)
{
    using v4 = typename Vec4<T>::type;
    using acc_t = typename Frag<T>::acc_t;
    constexpr int n_p = 64 * NT;
    constexpr int KC = n_p / 16;
    const int q = l >> 4, r = l & 15;
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
    const T* rowp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) rowp[t] = Hi + (int64_t)(16 * (NT * w + t) + r) * n_p + 4 * q;
    v4 cur[NT], nxt[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) cur[t] = *reinterpret_cast<const v4*>(rowp[t]);
    for (int K = 0; K < KC; ++K) {
        if (K + 1 < KC) {
#pragma unroll
            for (int t = 0; t < NT; ++t) nxt[t] = *reinterpret_cast<const v4*>(rowp[t] + 16 * (K + 1));
        }
        const v4 bv = *reinterpret_cast<const v4*>(ybuf + r * ldy + 16 * K + 4 * q);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = Frag<T>::mma(cur[t][s], bv[s], acc[t]);
        if (K + 1 < KC) {
#pragma unroll
            for (int t = 0; t < NT; ++t) cur[t] = nxt[t];
        }
    }
}

template <typename T, int NT>
struct SweepCtx {
    using acc_t = typename Frag<T>::acc_t;
    static constexpr int n_p = 64 * NT;
    static constexpr int ldy = n_p + 4;
    const SweepArgs& a;
    T* ybuf;
    T* Zs;
    const T* H;
    int w, l, q, col, b;
    bool bval;
    T g;

    __device__ int row_of(int t, int v) const { return 16 * (NT * w + t) + Frag<T>::drow(q, v); }
    __device__ T* zrow(int i) const { return Zs + (int64_t)i * 16 * n_p + col * n_p; }
    __device__ double vin(int i) const { return bval ? a.V[(int64_t)b * a.m + i] : 0.0; }

    // panel <- f_i + g * (sum of the given z rows); every lane fills the entries it owns
    __device__ void set_panel(int i, const acc_t (&zacc)[NT], bool with_acc, int zrow_a, int zrow_b) {
        const double vb = vin(i);
        const double* ci = a.c + (int64_t)i * n_p;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = row_of(t, v);
                T y = (T)(ci[k] * vb);
                if (with_acc) y += g * zacc[t][v];
                if (zrow_a >= 0) y += g * zrow(zrow_a)[pos<T>(k)];
                if (zrow_b >= 0) y += g * zrow(zrow_b)[pos<T>(k)];
                ybuf[col * ldy + pos<T>(k)] = y;
            }
        __syncthreads();
    }
    __device__ void put_panel(const acc_t (&u)[NT]) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) ybuf[col * ldy + pos<T>(row_of(t, v))] = u[t][v];
        __syncthreads();
    }
    __device__ void store_z(int i, const acc_t (&z)[NT]) {
        T* zr = zrow(i);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) zr[pos<T>(row_of(t, v))] = z[t][v];
    }
    // acc <- z_i + g * acc, written back over z_i
    __device__ void finish_back(int i, acc_t (&acc)[NT]) {
        T* zr = zrow(i);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = pos<T>(row_of(t, v));
                acc[t][v] = zr[p] + g * acc[t][v];
                zr[p] = acc[t][v];
            }
    }
    __device__ void currents(const acc_t (&u)[NT]) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = row_of(t, v);
                if (bval && k < a.n) a.Iout[(int64_t)b * a.n + k] = a.g_sense * (double)u[t][v];
            }
    }
};

template <typename T, int NT>
__global__ __launch_bounds__(256) void sweep_kernel(SweepArgs a)
{
    extern __shared__ __align__(32) unsigned char smem_raw[];
    using acc_t = typename Frag<T>::acc_t;
    using Ctx = SweepCtx<T, NT>;
    const int m = a.m, kt = m / 2;
    const int l = threadIdx.x & 63;
    Ctx x{a, reinterpret_cast<T*>(smem_raw),
          reinterpret_cast<T*>(a.Z) + (int64_t)blockIdx.x * m * 16 * Ctx::n_p,
          reinterpret_cast<const T*>(a.H), (int)(threadIdx.x >> 6), l, l >> 4, l & 15,
          16 * (int)blockIdx.x + (l & 15), false, (T)a.g_bl};
    x.bval = x.b < a.B;
    const int64_t blk = (int64_t)Ctx::n_p * Ctx::n_p;
    acc_t acc[NT];
    // forward, top chain
    if (kt > 0) {
        x.set_panel(0, acc, false, -1, -1);
        for (int i = 0; i < kt; ++i) {
            panel_product<T, NT>(acc, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.store_z(i, acc);
            if (i + 1 < kt) x.set_panel(i + 1, acc, true, -1, -1);
        }
    }
    // forward, bottom chain
    if (m - 1 > kt) {
        x.set_panel(m - 1, acc, false, -1, -1);
        for (int i = m - 1; i > kt; --i) {
            panel_product<T, NT>(acc, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.store_z(i, acc);
            if (i - 1 > kt) x.set_panel(i - 1, acc, true, -1, -1);
        }
    }
    // twist row
    x.set_panel(kt, acc, false, kt > 0 ? kt - 1 : -1, kt + 1 < m ? kt + 1 : -1);
    panel_product<T, NT>(acc, x.H + kt * blk, x.ybuf, Ctx::ldy, x.w, l);
    x.store_z(kt, acc);
    if (kt == m - 1) x.currents(acc);
    // back, upward
    if (kt > 0) {
        x.put_panel(acc);
        for (int i = kt - 1; i >= 0; --i) {
            acc_t u[NT];
            panel_product<T, NT>(u, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.finish_back(i, u);
            if (i > 0) x.put_panel(u);
        }
    }
    // back, downward
    if (kt + 1 < m) {
        {
            const T* zr = x.zrow(kt);
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[t][v] = zr[pos<T>(x.row_of(t, v))];
        }
        x.put_panel(acc);
        for (int i = kt + 1; i < m; ++i) {
            panel_product<T, NT>(acc, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.finish_back(i, acc);
            if (i == m - 1) x.currents(acc);
            else x.put_panel(acc);
        }
    }
}

// Word-line recovery and node-voltage output for one row block of 8 input
// vectors: T_i w = g_src V_i e_0 + Gam_i u_i by the Thomas recurrences
//   d'_0 = d_0, d'_j = d_j + fr_j d'_{j-1};  w_{n-1} = ip_{n-1} d'_{n-1},
//   w_j = ip_j (d'_j + g_wl w_{j+1}),
// each split over 32 lanes per vector as a scan of affine maps.
constexpr int kRecCols = 8;
constexpr int kRecLanes = 32;

__device__ inline void affine_compose(double& P, double& Q, double Pp, double Qp)
{
    // (P, Q) after (Pp, Qp): x -> P (Pp x + Qp) + Q
    Q = P * Qp + Q;
    P = P * Pp;
}

template <typename T>
__global__ __launch_bounds__(256) void recover_kernel(RecoverArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = a.n, m = a.m, n_p = a.n_p;
    double* ub = reinterpret_cast<double*>(smem_raw);       // [kRecCols][n]
    double* wb = ub + kRecCols * n;                           // [kRecCols][n]
    const int i = blockIdx.y;
    const int slab = blockIdx.x / 2, half = blockIdx.x % 2;
    const int c = threadIdx.x / kRecLanes, s = threadIdx.x % kRecLanes;
    const int colg = half * kRecCols + c;                    // column inside the 16-wide slab
    const int b = 16 * slab + colg;
    const bool bval = b < a.B;
    const T* Zi = reinterpret_cast<const T*>(a.Z) + ((int64_t)slab * m + i) * 16 * n_p;
    for (int e = threadIdx.x; e < kRecCols * n; e += blockDim.x) {
        const int cc = e / n, j = e % n;
        ub[e] = (double)Zi[(half * kRecCols + cc) * n_p + pos<T>(j)];
    }
    __syncthreads();
    const double* fr = a.fr + (int64_t)i * n;
    const double* ip = a.ip + (int64_t)i * n;
    const double* Gi = a.Gc + (int64_t)i * n;
    const double vin = bval ? a.V[(int64_t)b * m + i] : 0.0;
    const int seg = (n + kRecLanes - 1) / kRecLanes;
    const int j0 = s * seg, j1 = min(n, j0 + seg);
    double* u = ub + c * n;
    double* wv = wb + c * n;
    // forward: local map from d'_{j0-1} to d'_{j1-1}
    double P = 1.0, Q = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double d = Gi[j] * u[j] + (j == 0 ? a.g_src * vin : 0.0);
        Q = d + fr[j] * Q;
        P = fr[j] * P;
    }
    for (int off = 1; off < kRecLanes; off <<= 1) {          // inclusive scan, lane order
        const double Pp = __shfl_up(P, off, kRecLanes), Qp = __shfl_up(Q, off, kRecLanes);
        if (s >= off) affine_compose(P, Q, Pp, Qp);
    }
    double x = __shfl_up(Q, 1, kRecLanes);                    // d'_{j0-1}
    if (s == 0) x = 0.0;
    for (int j = j0; j < j1; ++j) {
        x = Gi[j] * u[j] + (j == 0 ? a.g_src * vin : 0.0) + fr[j] * x;
        wv[j] = x;                                            // d'_j
    }
    // backward: local map from w_{j1} to w_{j0}
    const double gw = a.g_wl;
    P = 1.0; Q = 0.0;
    for (int j = j1 - 1; j >= j0; --j) {
        const double f = (j == n - 1) ? 0.0 : ip[j] * gw;
        Q = ip[j] * wv[j] + f * Q;
        P = f * P;
    }
    for (int off = 1; off < kRecLanes; off <<= 1) {          // inclusive scan, reverse lane order
        const double Pp = __shfl_down(P, off, kRecLanes), Qp = __shfl_down(Q, off, kRecLanes);
        if (s + off < kRecLanes) affine_compose(P, Q, Pp, Qp);
    }
    x = __shfl_down(Q, 1, kRecLanes);                         // w_{j1}
    if (s == kRecLanes - 1) x = 0.0;
    for (int j = j1 - 1; j >= j0; --j) {
        const double f = (j == n - 1) ? 0.0 : ip[j] * gw;
        x = ip[j] * wv[j] + f * x;
        wv[j] = x;                                            // w_j
    }
    __syncthreads();
    if (a.node_v == nullptr) return;
    for (int e = threadIdx.x; e < kRecCols * 2 * n; e += blockDim.x) {
        const int cc = e / (2 * n), k = e % (2 * n);
        const int bb = 16 * slab + half * kRecCols + cc;
        if (bb < a.B) {
            const int j = k >> 1;
            a.node_v[(int64_t)bb * 2 * m * n + (int64_t)2 * i * n + k] = (k & 1) ? ub[cc * n + j] : wb[cc * n + j];
        }
    }
}

template <typename T, int NT>
hipError_t launch_sweep_nt(const SweepArgs& a, hipStream_t s)
{
    const size_t lds = 16 * (size_t)(64 * NT + 4) * sizeof(T);
    hipLaunchKernelGGL((sweep_kernel<T, NT>), dim3(a.nslab), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const SweepArgs& a, hipStream_t s)
{
    switch (a.n_p / 64) {
        case 1: return launch_sweep_nt<T, 1>(a, s);
        case 2: return launch_sweep_nt<T, 2>(a, s);
        case 3: return launch_sweep_nt<T, 3>(a, s);
        case 4: return launch_sweep_nt<T, 4>(a, s);
        case 5: return launch_sweep_nt<T, 5>(a, s);
        case 6: return launch_sweep_nt<T, 6>(a, s);
        case 7: return launch_sweep_nt<T, 7>(a, s);
        case 8: return launch_sweep_nt<T, 8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace xbk

hipError_t xbk_launch_sweep(const xbk::SweepArgs& a, bool fp32, hipStream_t s)
{
    return fp32 ? xbk::launch_sweep<float>(a, s) : xbk::launch_sweep<double>(a, s);
}

hipError_t xbk_launch_recover(const xbk::RecoverArgs& a, bool fp32, hipStream_t s)
{
    const size_t lds = 2 * xbk::kRecCols * (size_t)a.n * sizeof(double);
    dim3 grid(2 * a.nslab, a.m);
    if (fp32)
        hipLaunchKernelGGL(xbk::recover_kernel<float>, grid, dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(xbk::recover_kernel<double>, grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

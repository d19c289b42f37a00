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

template <typename T, int NT, bool IR>
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
    double dmax = 0.0, umax = 0.0;   // refinement: largest correction and solution entry seen

    __device__ int row_of(int t, int v) const { return 16 * (NT * w + t) + Frag<T>::drow(q, v); }
    __device__ int64_t rowoff(int i) const { return ((int64_t)blockIdx.x * a.m + i) * 16 * n_p + col * n_p; }
    __device__ T* zrow(int i) const { return Zs + (int64_t)i * 16 * n_p + col * n_p; }
    __device__ double vin(int i) const { return bval ? a.V[(int64_t)b * a.m + i] : 0.0; }

    // panel <- f_i + g * (z terms); f_i = V_i c_i, or the residual panel R_i when refining
    __device__ void set_panel(int i, const acc_t (&zacc)[NT], bool with_acc, int zrow_a, int zrow_b) {
        const bool from_r = IR && a.iter > 0;
        const double vb = from_r ? 0.0 : vin(i);
        const double* ci = a.c + (int64_t)i * n_p;
        const T* Ri = from_r ? reinterpret_cast<const T*>(a.R) + rowoff(i) : nullptr;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NT; ++t)
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
    // Row i of the back sweep is final in acc: write it where it belongs (over z_i, or
    // added to the float64 solution when refining) and emit the currents of row m-1.
    __device__ void settle(int i, const acc_t (&u)[NT]) {
        if (!IR) {
            store_z(i, u);
            if (i == a.m - 1) currents(u);
            return;
        }
        const int64_t ro = rowoff(i);
        const double* ui = a.Uin + ro;
        double* uo = a.Uout + ro;
#pragma unroll
        for (int t = 0; t < NT; ++t)
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
    __device__ void back_step(int i, acc_t (&acc)[NT]) {
        const T* zr = zrow(i);
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] = zr[pos<T>(row_of(t, v))] + g * acc[t][v];
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
    // Refinement bookkeeping for the slab: per input vector, stop when the error left after
    // this correction, estimated as |d| * min(1, |d| / |d_prev|), is <= tol * |u|.
    __device__ void decide(double* red) {
        double dm = dmax, um = umax;
        for (int off = 16; off < 64; off <<= 1) {
            dm = fmax(dm, __shfl_xor(dm, off));
            um = fmax(um, __shfl_xor(um, off));
        }
        __syncthreads();
        if (l < 16) {
            red[w * 16 + l] = dm;
            red[64 + w * 16 + l] = um;
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            double D = 0.0, U = 0.0;
            for (int k = 0; k < 4; ++k) {
                D = fmax(D, red[k * 16 + threadIdx.x]);
                U = fmax(U, red[64 + k * 16 + threadIdx.x]);
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

template <typename T, int NT, bool IR>
__global__ __launch_bounds__(256) void sweep_kernel(SweepArgs a)
{
    extern __shared__ __align__(32) unsigned char smem_raw[];
    using acc_t = typename Frag<T>::acc_t;
    using Ctx = SweepCtx<T, NT, IR>;
    if (IR && a.iter > 0 && a.slab_done[blockIdx.x]) return;
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
    if (IR) x.store_z(kt, acc);     // the downward back sweep restarts from this row
    x.settle(kt, acc);
    // back, upward
    if (kt > 0) {
        x.put_panel(acc);
        for (int i = kt - 1; i >= 0; --i) {
            acc_t u[NT];
            panel_product<T, NT>(u, x.H + i * blk, x.ybuf, Ctx::ldy, x.w, l);
            x.back_step(i, u);
            x.settle(i, u);
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
            x.back_step(i, acc);
            x.settle(i, acc);
            if (i < m - 1) x.put_panel(acc);
        }
    }
    if (IR) x.decide(reinterpret_cast<double*>(smem_raw + 16 * Ctx::ldy * sizeof(T)));
}

// Residual of the condensed system for the refinement, in float64:
//   r_i = V_i c_i - (E_i u_i - g_bl (u_{i-1} + u_{i+1})),
//   E_i u_i = Q_i u_i - Gam_i T_i^{-1} (Gam_i u_i)
// with T_i^{-1} applied by the same Thomas recurrences (affine scans) as the
// word-line recovery; rounded to float for the correction sweep.
constexpr int kResCols = 8;
constexpr int kResLanes = 32;

__device__ inline void affine_compose_d(double& P, double& Q, double Pp, double Qp)
{
    Q = P * Qp + Q;          // x -> P (Pp x + Qp) + Q
    P = P * Pp;
}

// Solve T_i w = d for one vector split over 32 lanes (contiguous segments),
// w overwriting d in LDS.  fr/ip: forward Thomas ratios and inverse pivots of T_i.
__device__ inline void tridiag_solve_lanes(double* d, const double* fr, const double* ip, double gw,
                                           int n, int s)
{
    const int seg = (n + kResLanes - 1) / kResLanes;
    const int j0 = s * seg, j1 = min(n, j0 + seg);
    double P = 1.0, Q = 0.0;
    for (int j = j0; j < j1; ++j) {
        Q = d[j] + fr[j] * Q;
        P = fr[j] * P;
    }
    for (int off = 1; off < kResLanes; off <<= 1) {
        const double Pp = __shfl_up(P, off, kResLanes), Qp = __shfl_up(Q, off, kResLanes);
        if (s >= off) affine_compose_d(P, Q, Pp, Qp);
    }
    double x = __shfl_up(Q, 1, kResLanes);
    if (s == 0) x = 0.0;
    for (int j = j0; j < j1; ++j) {
        x = d[j] + fr[j] * x;
        d[j] = x;
    }
    P = 1.0;
    Q = 0.0;
    for (int j = j1 - 1; j >= j0; --j) {
        const double f = (j == n - 1) ? 0.0 : ip[j] * gw;
        Q = ip[j] * d[j] + f * Q;
        P = f * P;
    }
    for (int off = 1; off < kResLanes; off <<= 1) {
        const double Pp = __shfl_down(P, off, kResLanes), Qp = __shfl_down(Q, off, kResLanes);
        if (s + off < kResLanes) affine_compose_d(P, Q, Pp, Qp);
    }
    x = __shfl_down(Q, 1, kResLanes);
    if (s == kResLanes - 1) x = 0.0;
    for (int j = j1 - 1; j >= j0; --j) {
        const double f = (j == n - 1) ? 0.0 : ip[j] * gw;
        x = ip[j] * d[j] + f * x;
        d[j] = x;
    }
}

__global__ __launch_bounds__(256) void residual_kernel(ResidualArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = a.n, m = a.m, n_p = a.n_p;
    const int i = blockIdx.y;
    const int slab = blockIdx.x / 2, half = blockIdx.x % 2;
    if (a.slab_done[slab]) return;
    double* wb = reinterpret_cast<double*>(smem_raw);             // [kResCols][n]
    const int c = threadIdx.x / kResLanes, s = threadIdx.x % kResLanes;
    const int colg = half * kResCols + c;
    const int b = 16 * slab + colg;
    const double* Gi = a.Gc + (int64_t)i * n;
    const double* Ui = a.U + (((int64_t)slab * m + i) * 16 + colg) * n_p;
    double* w = wb + c * n;
    for (int j = s; j < n; j += kResLanes) w[j] = Gi[j] * Ui[j];
    __syncthreads();
    tridiag_solve_lanes(w, a.fr + (int64_t)i * n, a.ip + (int64_t)i * n, a.g_wl, n, s);
    __syncthreads();
    const double vb = (b < a.B) ? a.V[(int64_t)b * m + i] : 0.0;
    const double* ci = a.c + (int64_t)i * n_p;
    const double* qi = a.q + (int64_t)i * n;
    const double* Uup = (i > 0) ? Ui - 16 * (int64_t)n_p : nullptr;
    const double* Udn = (i + 1 < m) ? Ui + 16 * (int64_t)n_p : nullptr;
    float* Ri = reinterpret_cast<float*>(a.R) + (((int64_t)slab * m + i) * 16 + colg) * n_p;
    for (int j = s; j < n; j += kResLanes) {
        double r = ci[j] * vb - (qi[j] * Ui[j] - Gi[j] * w[j]);
        if (Uup) r += a.g_bl * Uup[j];
        if (Udn) r += a.g_bl * Udn[j];
        Ri[j] = (float)r;
    }
    for (int j = n + s; j < n_p; j += kResLanes) Ri[j] = 0.0f;      // padding stays zero
}

// Word-line recovery and node-voltage output for one row block of 8 input
// vectors: T_i w = g_src V_i e_0 + Gam_i u_i, solved by the Thomas recurrences
// split over 32 lanes per vector (tridiag_solve_lanes), then written out in
// the paper's interleaved node order with coalesced stores.
constexpr int kRecCols = kResCols;

template <typename T>
__global__ __launch_bounds__(256) void recover_kernel(RecoverArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = a.n, m = a.m, n_p = a.n_p;
    double* ub = reinterpret_cast<double*>(smem_raw);       // [kRecCols][n]
    double* wb = ub + kRecCols * n;                           // [kRecCols][n]
    const int i = blockIdx.y;
    const int slab = blockIdx.x / 2, half = blockIdx.x % 2;
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
    double* u = ub + c * n;
    double* wv = wb + c * n;
    for (int j = s; j < n; j += kResLanes) wv[j] = Gi[j] * u[j] + (j == 0 ? a.g_src * vin : 0.0);
    __syncthreads();
    tridiag_solve_lanes(wv, a.fr + (int64_t)i * n, a.ip + (int64_t)i * n, a.g_wl, n, s);
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

template <typename T, int NT, bool IR>
hipError_t launch_sweep_nt(const SweepArgs& a, hipStream_t s)
{
    const size_t lds = 16 * (size_t)(64 * NT + 4) * sizeof(T) + (IR ? 128 * sizeof(double) : 0);
    hipLaunchKernelGGL((sweep_kernel<T, NT, IR>), dim3(a.nslab), dim3(256), lds, s, a);
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
    const size_t lds = xbk::kResCols * (size_t)a.n * sizeof(double);
    hipLaunchKernelGGL(xbk::residual_kernel, dim3(2 * a.nslab, a.m), dim3(256), lds, s, a);
    return hipGetLastError();
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

// Block LU of the condensed bit-line system (the decomposition of Sec. II.C,
// done over row blocks).
//
// After condensation the bit-line voltages satisfy the block-tridiagonal
// system  E_i u_i - g_bl (u_{i-1} + u_{i+1}) = V_i c_i.  Its block LU
// (block-Thomas) has the pivot blocks
//     S_0 = E_0,   S_t = E_t - g_bl^2 S_{t-1}^{-1},
// and the substitution only needs H_t = S_t^{-1}, which this file computes,
// sequentially in t, overwriting E_t with H_t in place.
//
// Each inverse is an in-place blocked Gauss-Jordan elimination on 64 x 64
// tiles (no row exchanges: every S_t is symmetric positive definite, a
// Schur complement of the SPD nodal matrix).  For pivot block k with
// P = S[k][k]:
//     S[I][J] -= S[I][k] (P^{-1} S[k][J])      I != k, J != k
//     S[k][J]  = P^{-1} S[k][J]                J != k
//     S[I][k]  = -S[I][k] P^{-1}                I != k
//     S[k][k]  = P^{-1}
// One kernel launch per pivot block (the launch boundary is the only
// grid-wide synchronisation); workgroup (I, J) updates tile (I, J) with two
// 64^3 MFMA products.  The workgroup that owns the next pivot tile inverts
// it before exiting, so P^{-1} is ready when the next launch starts; the
// last launch of step t also forms S_{t+1} = E_{t+1} - g_bl^2 H_t tile by
// tile and inverts its first pivot tile.
#include "common.h"

namespace xbk {

constexpr int kLd = kTile + 4;          // LDS row pitch (elements) for operand tiles
constexpr int kLdP = kTile + 1;         // LDS row pitch for the pivot inversion

// acc[C] += A(16w.. rows, 64) * B(64, 16C.. cols); sA row-major CPR, sB = B^T, CPR on k.
template <typename T>
__device__ inline void tile_mma(typename Frag<T>::acc_t (&acc)[4], const T* sA, const T* sB, int w, int l)
{
    const int q = l >> 4, r = l & 15;
#pragma unroll
    for (int K = 0; K < 4; ++K) {
        T av[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) av[t] = sA[(16 * w + r) * kLd + 16 * K + 4 * q + t];
#pragma unroll
        for (int C = 0; C < 4; ++C) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[C] = Frag<T>::mma(av[t], sB[(16 * C + r) * kLd + 16 * K + 4 * q + t], acc[C]);
        }
    }
}

// Stage a 64x64 tile of a CPR matrix as an A operand (same CPR order), scaled by s.
template <typename T>
__device__ inline void stage_A(T* sA, const T* M, int ld, int r0, int c0, T s)
{
    for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
        const int r = e / kTile, p = e % kTile;
        sA[r * kLd + p] = s * M[(int64_t)(r0 + r) * ld + c0 + p];
    }
}

// Stage a 64x64 tile of a CPR matrix as a B operand: sB[col][slot(k)] = M[k][col].
template <typename T>
__device__ inline void stage_B(T* sB, const T* M, int ld, int r0, int c0)
{
    for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
        const int kk = e / kTile, p = e % kTile;       // global position p holds column 16(p/16)+slot(p%16)
        const int cc = (p & ~15) + Frag<T>::slot(p & 15);
        sB[cc * kLd + (kk & ~15) + Frag<T>::slot(kk & 15)] = M[(int64_t)(r0 + kk) * ld + c0 + p];
    }
}

// Element (row, col) of the output sub-tile held by lane l, item v, of wave w.
__device__ inline int out_row(int w, int l, int v, bool f64) { return 16 * w + (f64 ? ((l >> 4) + 4 * v) : (4 * (l >> 4) + v)); }

template <typename T>
__device__ inline void load_acc(typename Frag<T>::acc_t (&acc)[4], const T* M, int ld, int r0, int c0, int w, int l)
{
    constexpr bool f64 = sizeof(T) == 8;
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            acc[C][v] = M[cpr<T>(r0 + out_row(w, l, v, f64), c0 + 16 * C + (l & 15), ld)];
}

template <typename T>
__device__ inline void store_acc(const typename Frag<T>::acc_t (&acc)[4], T* M, int ld, int r0, int c0, int w, int l)
{
    constexpr bool f64 = sizeof(T) == 8;
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            M[cpr<T>(r0 + out_row(w, l, v, f64), c0 + 16 * C + (l & 15), ld)] = acc[C][v];
}

// In-place Gauss-Jordan inverse of the 64x64 SPD tile held in acc (C layout);
// result written row-major CPR to Pout.  Raises kErrPivot on a bad pivot.
template <typename T>
__device__ void invert_tile(const typename Frag<T>::acc_t (&acc)[4], T* sP, T* Pout, int* flags, int w, int l)
{
    constexpr bool f64 = sizeof(T) == 8;
    __syncthreads();
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) sP[out_row(w, l, v, f64) * kLdP + 16 * C + (l & 15)] = acc[C][v];
    __syncthreads();
    const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
    bool bad = false;
    for (int p = 0; p < kTile; ++p) {
        const T d = sP[p * kLdP + p];
        const T arp = sP[r * kLdP + p];
        T prow[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) prow[c] = sP[p * kLdP + c0 + c];
        __syncthreads();
        bad |= !(d > (T)0) || !isfinite(d);
        const T inv = (T)1 / d;
        if (r == p) {
#pragma unroll
            for (int c = 0; c < 16; ++c) sP[p * kLdP + c0 + c] = (c0 + c == p) ? inv : prow[c] * inv;
        } else {
            const T f = arp * inv;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                T* x = &sP[r * kLdP + c0 + c];
                *x = (c0 + c == p) ? -f : *x - f * prow[c];
            }
        }
        __syncthreads();
    }
    if (bad) atomicOr(flags + kErrPivot, 1);
    for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
        const int rr = e / kTile, cc = e % kTile;
        Pout[cpr<T>(rr, cc, kTile)] = sP[rr * kLdP + cc];
    }
}

// S_t(r, c) for block t: E_t - g^2 H_{t-1} on the n x n part, identity on the padding.
template <typename T>
__device__ inline T form_S(T e, T h, double g2, int r, int c, int n)
{
    if (r < n && c < n) return e - (T)g2 * h;
    return (r == c) ? (T)1 : (T)0;
}

// Chain step 0: S_0 = E_0 (identity padding) into S[0]; pivot tile (0,0) inverted into P[0].
template <typename T>
__global__ __launch_bounds__(256) void gj_init_kernel(GJArgs a)
{
    __shared__ T sP[kTile * kLdP];
    const int I = blockIdx.x / a.nb, J = blockIdx.x % a.nb;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const T* E0 = reinterpret_cast<const T*>(a.H);
    T* S = reinterpret_cast<T*>(a.S0);
    typename Frag<T>::acc_t acc[4];
    load_acc<T>(acc, E0, a.n_p, 64 * I, 64 * J, w, l);
    constexpr bool f64 = sizeof(T) == 8;
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            acc[C][v] = form_S<T>(acc[C][v], (T)0, 0.0, 64 * I + out_row(w, l, v, f64),
                                  64 * J + 16 * C + (l & 15), a.n);
    store_acc<T>(acc, S, a.n_p, 64 * I, 64 * J, w, l);
    if (I == 0 && J == 0) invert_tile<T>(acc, sP, reinterpret_cast<T*>(a.P0), a.flags, w, l);
}

// Pivot block k of chain step t.  g = t*nb + k selects the ping-pong buffers.
template <typename T>
__global__ __launch_bounds__(256) void gj_step_kernel(GJArgs a, int t, int k)
{
    __shared__ T sA[kTile * kLd];
    __shared__ T sB[kTile * kLd];
    const int nb = a.nb, n_p = a.n_p;
    const int I = blockIdx.x / nb, J = blockIdx.x % nb;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t g = (int64_t)t * nb + k;
    const T* Sin = reinterpret_cast<const T*>((g & 1) ? a.S1 : a.S0);
    T* Sout = reinterpret_cast<T*>((g & 1) ? a.S0 : a.S1);
    const T* Pin = reinterpret_cast<const T*>((g & 1) ? a.P1 : a.P0);
    T* Pout = reinterpret_cast<T*>((g & 1) ? a.P0 : a.P1);
    const bool last = (k == nb - 1);
    using acc_t = typename Frag<T>::acc_t;
    acc_t acc[4];
#pragma unroll
    for (int C = 0; C < 4; ++C) acc[C] = acc_t{0, 0, 0, 0};

    const int r0 = 64 * I, c0 = 64 * J, pk = 64 * k;
    if (I != k && J != k) {
        stage_A<T>(sA, Pin, kTile, 0, 0, (T)1);
        stage_B<T>(sB, Sin, n_p, pk, c0);
        __syncthreads();
        tile_mma<T>(acc, sA, sB, w, l);                 // X = P^{-1} S[k][J]
        __syncthreads();
        constexpr bool f64 = sizeof(T) == 8;
#pragma unroll
        for (int C = 0; C < 4; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) {               // X as the next B operand: sB[col][slot(k)]
                const int kk = out_row(w, l, v, f64);
                sB[(16 * C + (l & 15)) * kLd + (kk & ~15) + Frag<T>::slot(kk & 15)] = acc[C][v];
            }
        stage_A<T>(sA, Sin, n_p, r0, pk, (T)-1);
        load_acc<T>(acc, Sin, n_p, r0, c0, w, l);
        __syncthreads();
        tile_mma<T>(acc, sA, sB, w, l);                 // S[I][J] - S[I][k] X
    } else if (I == k && J != k) {
        stage_A<T>(sA, Pin, kTile, 0, 0, (T)1);
        stage_B<T>(sB, Sin, n_p, pk, c0);
        __syncthreads();
        tile_mma<T>(acc, sA, sB, w, l);                 // P^{-1} S[k][J]
    } else if (I != k && J == k) {
        stage_A<T>(sA, Sin, n_p, r0, pk, (T)-1);
        stage_B<T>(sB, Pin, kTile, 0, 0);
        __syncthreads();
        tile_mma<T>(acc, sA, sB, w, l);                 // -S[I][k] P^{-1}
    } else {
        load_acc<T>(acc, Pin, kTile, 0, 0, w, l);       // P^{-1}
    }

    T* sP = sA;   // operand tiles are dead from here on; reuse for the pivot inversion
    if (!last) {
        store_acc<T>(acc, Sout, n_p, r0, c0, w, l);
        if (I == k + 1 && J == k + 1) invert_tile<T>(acc, sP, Pout, a.flags, w, l);
        return;
    }
    // Last pivot block: acc holds H_t[I][J].  Store it over E_t, then form S_{t+1}.
    T* Ht = reinterpret_cast<T*>(a.H) + (int64_t)t * n_p * n_p;
    store_acc<T>(acc, Ht, n_p, r0, c0, w, l);
    if (t + 1 >= a.m) return;
    const T* En = Ht + (int64_t)n_p * n_p;
    constexpr bool f64 = sizeof(T) == 8;
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = r0 + out_row(w, l, v, f64), cc = c0 + 16 * C + (l & 15);
            acc[C][v] = form_S<T>(En[cpr<T>(rr, cc, n_p)], acc[C][v], a.g2, rr, cc, a.n);
        }
    store_acc<T>(acc, Sout, n_p, r0, c0, w, l);
    if (I == 0 && J == 0) invert_tile<T>(acc, sP, Pout, a.flags, w, l);
}

template <typename T>
hipError_t launch_factor(const GJArgs& a, hipStream_t s)
{
    const int tiles = a.nb * a.nb;
    hipLaunchKernelGGL(gj_init_kernel<T>, dim3(tiles), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int t = 0; t < a.m; ++t)
        for (int k = 0; k < a.nb; ++k) {
            hipLaunchKernelGGL(gj_step_kernel<T>, dim3(tiles), dim3(256), 0, s, a, t, k);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace xbk

hipError_t xbk_launch_factor(const xbk::GJArgs& a, bool fp32, hipStream_t s)
{
    return fp32 ? xbk::launch_factor<float>(a, s) : xbk::launch_factor<double>(a, s);
}

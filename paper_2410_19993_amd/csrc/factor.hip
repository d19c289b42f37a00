// Block LU of the condensed bit-line system (the decomposition of Sec. II.C,
// done over row blocks), in twisted ("burn at both ends") order.
//
// After condensation the bit-line voltages satisfy the block-tridiagonal
// system  E_i u_i - g_bl (u_{i-1} + u_{i+1}) = V_i c_i.  Its block LU from the
// top has pivots S_0 = E_0, S_i = E_i - g_bl^2 S_{i-1}^{-1}; from the bottom,
// S'_{m-1} = E_{m-1}, S'_i = E_i - g_bl^2 S'_{i+1}^{-1}.  Running the top
// recurrence on rows 0..kt-1 and the bottom one on rows m-1..kt+1 at the same
// time, with kt = m/2, leaves the twist block
//     K = E_kt - g_bl^2 S_{kt-1}^{-1} - g_bl^2 S'_{kt+1}^{-1}
// and halves the sequential chain.  This file stores H_i = (pivot of row i)^{-1}
// over E_i: S_i^{-1} above kt, S'_i^{-1} below, K^{-1} at kt.
//
// Each inverse is an in-place blocked Gauss-Jordan elimination on 64 x 64
// tiles (no row exchanges: every pivot block is symmetric positive definite,
// a Schur complement of the SPD nodal matrix).  For pivot block k, P = S[k][k]:
//     S[I][J] -= S[I][k] (P^{-1} S[k][J])      I != k, J != k
//     S[k][J]  = P^{-1} S[k][J]                J != k
//     S[I][k]  = -S[I][k] P^{-1}                I != k
//     S[k][k]  = P^{-1}
// One launch per pivot block serves both chains (the launch boundary is the
// grid-wide synchronisation); workgroup (chain, I, J) updates tile (I, J).
// The workgroup owning the next pivot tile inverts it before exiting, and
// the last launch of a row forms the chain's next pivot block tile by tile.
#include <type_traits>

#include "common.h"

namespace xbk {

constexpr int kLd = kTile + 4;          // LDS pitch (elements) of operand tiles
constexpr int kTT = kTile * kTile;

template <typename T>
__device__ inline int out_row(int w, int l, int v)
{
    return 16 * w + Frag<T>::drow(l >> 4, v);
}

// Orders one wave's own LDS accesses (the wave's lanes exchange values through LDS).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// acc[C] += A(rows 16w.., 64) * B(64, cols 16C..); sA row-major CPR, sB = B^T (CPR on k).
template <typename T>
__device__ inline void tile_mma(typename Frag<T>::acc_t (&acc)[4], const T* sA, const T* sB, int w, int l)
{
    const int q = l >> 4, r = l & 15;
#pragma unroll
    for (int K = 0; K < 4; ++K) {
        T av[4], bv[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) av[t] = sA[(16 * w + r) * kLd + 16 * K + 4 * q + t];
#pragma unroll
        for (int C = 0; C < 4; ++C)
#pragma unroll
            for (int t = 0; t < 4; ++t) bv[C][t] = sB[(16 * C + r) * kLd + 16 * K + 4 * q + t];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int C = 0; C < 4; ++C) acc[C] = Frag<T>::mma(av[t], bv[C][t], acc[C]);
    }
}

// A-operand fragments of a 64x64 tile straight from memory into registers: rows
// r0 + 16w + (l & 15), columns c0 + 16K + 4(l >> 4) + t of chunk K.  The memory
// layout (row-major, columns permuted inside each 16-chunk) puts a lane's four values
// of a chunk next to each other, as in an LDS-staged A tile.
template <typename T>
__device__ inline void fetch_afrag(T (&av)[4][4], const T* __restrict__ M, int ld, int r0, int c0, int w, int l)
{
    const T* p = M + (int64_t)(r0 + 16 * w + (l & 15)) * ld + c0 + 4 * (l >> 4);
#pragma unroll
    for (int K = 0; K < 4; ++K)
#pragma unroll
        for (int t = 0; t < 4; ++t) av[K][t] = p[16 * K + t];
}

// acc[C] += s A(rows 16w.., 64) * B(64, cols 16C..) with A's fragments in registers
// (fetch_afrag) and B as for tile_mma: the same products in the same order as
// tile_mma on an A tile staged with the scale s.
template <typename T>
__device__ inline void tile_mma_r(typename Frag<T>::acc_t (&acc)[4], const T (&av)[4][4], T s, const T* sB, int w,
                                  int l)
{
    const int q = l >> 4, r = l & 15;
#pragma unroll
    for (int K = 0; K < 4; ++K) {
        T bv[4][4];
#pragma unroll
        for (int C = 0; C < 4; ++C)
#pragma unroll
            for (int t = 0; t < 4; ++t) bv[C][t] = sB[(16 * C + r) * kLd + 16 * K + 4 * q + t];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const T x = s * av[K][t];
#pragma unroll
            for (int C = 0; C < 4; ++C) acc[C] = Frag<T>::mma(x, bv[C][t], acc[C]);
        }
    }
}

// Operand staging is split into a fetch (global -> registers, 16 values per
// thread, row-contiguous across a wave) and a put (registers -> LDS), so that a
// workgroup can issue every global load of a launch before waiting on any.
constexpr int kPer = kTT / 256;

template <typename T>
__device__ inline void fetch_tile(T (&v)[kPer], const T* __restrict__ M, int ld, int r0, int c0)
{
    const int p = threadIdx.x & 63, rb = threadIdx.x >> 6;
#pragma unroll
    for (int it = 0; it < kPer; ++it) v[it] = M[(int64_t)(r0 + rb + 4 * it) * ld + c0 + p];
}

// A operand: same CPR order as in memory, scaled by s.
template <typename T>
__device__ inline void put_A(T* sA, const T (&v)[kPer], T s)
{
    const int p = threadIdx.x & 63, rb = threadIdx.x >> 6;
#pragma unroll
    for (int it = 0; it < kPer; ++it) sA[(rb + 4 * it) * kLd + p] = s * v[it];
}

// B operand: sB[col][slot(k)] = M[k][col] (memory position p holds column 16(p/16)+slot(p%16)).
template <typename T>
__device__ inline void put_B(T* sB, const T (&v)[kPer])
{
    const int p = threadIdx.x & 63, rb = threadIdx.x >> 6;
    const int cc = (p & ~15) + Frag<T>::slot(p & 15);
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
        const int kk = rb + 4 * it;
        sB[cc * kLd + (kk & ~15) + Frag<T>::slot(kk & 15)] = v[it];
    }
}

template <typename T>
__device__ inline void load_acc(typename Frag<T>::acc_t (&acc)[4], const T* __restrict__ M, int ld,
                                int r0, int c0, int w, int l)
{
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            acc[C][v] = M[cpr<T>(r0 + out_row<T>(w, l, v), c0 + 16 * C + (l & 15), ld)];
}

template <typename T>
__device__ inline void store_acc(const typename Frag<T>::acc_t (&acc)[4], T* M, int ld, int r0, int c0,
                                 int w, int l)
{
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            M[cpr<T>(r0 + out_row<T>(w, l, v), c0 + 16 * C + (l & 15), ld)] = acc[C][v];
}

// Gauss-Jordan inverse of the 64x64 SPD tile held in acc (MFMA output layout),
// written row-major CPR to Pout, four pivots per step.  Thread t keeps row t/4,
// columns 16(t%4)..+15 in registers.  For the pivot block D of rows and columns
// p..p+3, with R the pivot rows and C the pivot columns,
//     D <- D^-1,  R <- D^-1 R,  C <- -C D^-1,  A <- A - C D^-1 R,
// the pivot rows and columns go through double-buffered LDS (one barrier per step),
// and every thread inverts the 4x4 pivot block itself by scalar Gauss-Jordan (whose
// pivots are the elimination's scalar pivots).  A pivot that is not positive and
// finite raises kErrPivot.  `valid` pivots of the tile lie inside the n x n block
// (the rest are the identity padding); the smallest of them is folded into the
// plan's diagnostics.
template <typename T>
__device__ void invert_tile(const typename Frag<T>::acc_t (&acc)[4], T* lds, T* Pout, int* flags,
                            unsigned long long* diag, int valid, int w, int l, int* tbad, T* Pout2 = nullptr)
{
    T* sP = lds;                         // [64][kLd] staging of the tile
    __syncthreads();
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) sP[out_row<T>(w, l, v) * kLd + 16 * C + (l & 15)] = acc[C][v];
    __syncthreads();
    const int r = threadIdx.x >> 2, cbk = threadIdx.x & 3, c0 = cbk * 16;
    T a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = sP[r * kLd + c0 + c];
    __syncthreads();                     // the staging area becomes the pivot buffers
    T* rowb = lds;                       // [2][4][64] pivot rows
    T* colb = lds + 2 * 4 * kTile;       // [2][4][64] pivot columns
    bool bad = false;
    double dmin = __builtin_inf();
    for (int p = 0; p < kTile; p += 4) {
        const int buf = (p >> 2) & 1;
        T* rb = rowb + buf * 4 * kTile;
        T* cb = colb + buf * 4 * kTile;
        const int ir = r - p;                           // pivot row index, if 0..3
        const bool prow = ir >= 0 && ir < 4;
        const int cp = p >> 4, op = p & 15;             // chunk and offset of the pivot columns
        if (prow) {
#pragma unroll
            for (int c = 0; c < 16; ++c) rb[ir * kTile + c0 + c] = a[c];
        }
        if (cbk == cp) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                T v = a[0];
#pragma unroll
                for (int c = 1; c < 16; ++c) v = (c == op + j) ? a[c] : v;
                cb[j * kTile + r] = v;
            }
        }
        __syncthreads();
        // D^-1 by scalar Gauss-Jordan on the 4x4 block (its pivots are the scalar pivots)
        T D[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) D[i][j] = rb[i * kTile + p + j];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T d = D[k][k];
            bad |= !(d > (T)0) || !isfinite(d);
            if (p + k < valid) dmin = ((double)d < dmin || d != d) ? (double)d : dmin;
            const T inv = (T)1 / d;
            T rowk[4], colk[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                rowk[j] = D[k][j];
                colk[j] = D[j][k];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    T x;
                    if (i == k && j == k) x = inv;
                    else if (i == k) x = rowk[j] * inv;
                    else if (j == k) x = -colk[i] * inv;
                    else x = D[i][j] - colk[i] * inv * rowk[j];
                    D[i][j] = x;
                }
        }
        // this row's pivot-column entries C[r][i] (own registers or LDS) and F = C D^-1
        T Cr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) Cr[i] = cb[i * kTile + r];
        T F[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) F[j] = Cr[0] * D[0][j] + Cr[1] * D[1][j] + Cr[2] * D[2][j] + Cr[3] * D[3][j];
        T Dr[4];                                        // row ir of D^-1 (pivot rows)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T v = D[0][j];
#pragma unroll
            for (int i = 1; i < 4; ++i) v = (ir == i) ? D[i][j] : v;
            Dr[j] = v;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int col = c0 + c, jc = col - p;
            const bool pcol = jc >= 0 && jc < 4;
            const T R0 = rb[0 * kTile + col], R1 = rb[1 * kTile + col], R2 = rb[2 * kTile + col],
                    R3 = rb[3 * kTile + col];
            const T upd = a[c] - (F[0] * R0 + F[1] * R1 + F[2] * R2 + F[3] * R3);
            const T prw = Dr[0] * R0 + Dr[1] * R1 + Dr[2] * R2 + Dr[3] * R3;
            T fj = F[0], dj = Dr[0];
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                fj = (jc == j) ? F[j] : fj;
                dj = (jc == j) ? Dr[j] : dj;
            }
            a[c] = prow ? (pcol ? dj : prw) : (pcol ? -fj : upd);
        }
    }
    if (bad) {
        atomicOr(flags + kErrPivot, 1);
        if (tbad) atomicOr(tbad, 1);
    }
    if (threadIdx.x == 0 && valid > 0) atomicMin(diag + kDiagMinPivot, pivot_key(dmin));
#pragma unroll
    for (int c = 0; c < 16; ++c) Pout[cpr<T>(r, c0 + c, kTile)] = a[c];
    if (Pout2) {
#pragma unroll
        for (int c = 0; c < 16; ++c) Pout2[cpr<T>(r, c0 + c, kTile)] = a[c];
    }
}

// A 64x64 tile held in the accumulator layout (row out_row(w, l, v), column 16C + (l & 15))
// into an operand area: as the A operand (row-major, columns in chunk order) or as the
// B operand (stored transposed, rows in chunk order).
template <typename T>
__device__ inline void acc_to_A(T* sA, const typename Frag<T>::acc_t (&x)[4], int w, int l)
{
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) sA[out_row<T>(w, l, v) * kLd + 16 * C + Frag<T>::slot(l & 15)] = x[C][v];
}

template <typename T>
__device__ inline void acc_to_B(T* sB, const typename Frag<T>::acc_t (&x)[4], int w, int l)
{
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = out_row<T>(w, l, v);
            sB[(16 * C + (l & 15)) * kLd + (kk & ~15) + Frag<T>::slot(kk & 15)] = x[C][v];
        }
}

constexpr double kTileNsDone = 2.5e-7;  // largest |Q| entry accepted

// Inverse of the pivot tile P (in acc) by one third-order Newton-Schulz round on the
// matrix cores, from the chain's inverse Wk of the same tile one row earlier,
// corrected to first order in the change of the tile with that inverse taken as its
// diagonal (Pk: the tile one row earlier; consecutive rows' pivot tiles differ
// little, as the pivot blocks do):
//     X0 = Wk + diag(P)^-1 - diag(Pk)^-1 - D offdiag(P - Pk) D,   D = diag(Pk)^-1,
//     Q = I - X0 P,   Y = Q X0,   X = X0 + Y + Q Y,   I - X P = Q^3.
// Accepted when every |Q| entry is <= 2.5e-7, so ||Q||_inf <= 1.6e-5 and
// ||I - X P||_inf <= 4.1e-15 (on the 256 x 256 tiles of the tiles workload the
// corrected start leaves |Q| <= 9e-9, so X ends at rounding level; uncorrected it
// would leave |Q| near 2e-4, and the test would fail every tile): X goes to Pout and
// Wk, P to Pk, and the call returns true.  Otherwise (NaN included) it writes nothing
// and returns false after the first product, and the caller eliminates.  Three
// 64 x 64 x 64 products against the 16 dependent elimination steps; no pivot is
// examined on this path.  sA, sB: the workgroup's two operand areas.
template <typename T>
__device__ bool ns_tile_inverse(const typename Frag<T>::acc_t (&P)[4], T* Wk, T* Pk, T* sA, T* sB, T* Pout, int w,
                                int l)
{
    using acc_t = typename Frag<T>::acc_t;
    __shared__ double wmx[4];
    acc_t x[4], q[4], t[4];
    {
        acc_t pp[4];
        T dpr[4], dpc[4];
        load_acc<T>(x, Wk, kTile, 0, 0, w, l);
        load_acc<T>(pp, Pk, kTile, 0, 0, w, l);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = out_row<T>(w, l, v);
            dpr[v] = Pk[cpr<T>(rr, rr, kTile)];
        }
#pragma unroll
        for (int C = 0; C < 4; ++C) {
            const int cc = 16 * C + (l & 15);
            dpc[C] = Pk[cpr<T>(cc, cc, kTile)];
        }
#pragma unroll
        for (int C = 0; C < 4; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (out_row<T>(w, l, v) == 16 * C + (l & 15))
                    x[C][v] += (T)1 / P[C][v] - (T)1 / dpr[v];
                else
                    x[C][v] -= (P[C][v] - pp[C][v]) / (dpr[v] * dpc[C]);
            }
    }
    __syncthreads();                                    // the operand areas are free
    acc_to_A<T>(sA, x, w, l);
    acc_to_B<T>(sB, P, w, l);
    __syncthreads();
#pragma unroll
    for (int C = 0; C < 4; ++C) q[C] = acc_t{0, 0, 0, 0};
    tile_mma<T>(q, sA, sB, w, l);                       // X0 P
    double mx = 0.0;
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            q[C][v] = (T)(out_row<T>(w, l, v) == 16 * C + (l & 15) ? 1 : 0) - q[C][v];
            mx = nan_max(mx, fabs((double)q[C][v]));
        }
    for (int off = 32; off > 0; off >>= 1) mx = nan_max(mx, __shfl_xor(mx, off));
    if (l == 0) wmx[w] = mx;
    __syncthreads();                                    // X0 and P read; wmx written
    const double nu = nan_max(nan_max(wmx[0], wmx[1]), nan_max(wmx[2], wmx[3]));
    if (!(nu <= kTileNsDone)) return false;             // the same answer in every wave
    acc_to_A<T>(sA, q, w, l);
    acc_to_B<T>(sB, x, w, l);
    __syncthreads();
#pragma unroll
    for (int C = 0; C < 4; ++C) t[C] = acc_t{0, 0, 0, 0};
    tile_mma<T>(t, sA, sB, w, l);                       // Y = Q X0
    __syncthreads();                                    // X0 in sB read
    acc_to_B<T>(sB, t, w, l);
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) x[C][v] += t[C][v];
    __syncthreads();
    tile_mma<T>(x, sA, sB, w, l);                       // X = X0 + Y + Q Y
    store_acc<T>(x, Pout, kTile, 0, 0, w, l);
    store_acc<T>(x, Wk, kTile, 0, 0, w, l);             // Wk and Pk were read into registers
    store_acc<T>(P, Pk, kTile, 0, 0, w, l);
    return true;
}

// The pivot tile in acc inverted into Pout.  NS (a batch with warm-start slots): by the
// Newton-Schulz round when `warm` (the slots hold the chain's inverse of this tile and
// the tile one row earlier) and it is accepted, else by elimination; either way the
// slots then hold this row's inverse and tile.  W: the slots of the tile (inverse; the
// tile nb tiles on).  Without NS: elimination only, W unused.
template <typename T, bool NS>
__device__ void invert_pivot(const typename Frag<T>::acc_t (&acc)[4], T* sA, T* sB, T* Pout, T* W, int nb,
                             bool warm, int* flags, unsigned long long* diag, int valid, int w, int l, int* tbad)
{
    if constexpr (NS) {
        T* const Pk = W + (int64_t)nb * kTile * kTile;
        if (warm && ns_tile_inverse<T>(acc, W, Pk, sA, sB, Pout, w, l)) return;
        invert_tile<T>(acc, sA, Pout, flags, diag, valid, w, l, tbad, W);
        store_acc<T>(acc, Pk, kTile, 0, 0, w, l);
    } else {
        invert_tile<T>(acc, sA, Pout, flags, diag, valid, w, l, tbad);
    }
}

// Pivot block of a row: E_row - g^2 (H_a + H_b) on the n x n part (a, b < 0: absent),
// identity on the padding.
template <typename T>
__device__ inline T form_elem(const T* E, const T* Ha, const T* Hb, int64_t off, double g2, int r, int c, int n)
{
    if (r >= n || c >= n) return (r == c) ? (T)1 : (T)0;
    T s = E[off];
    if (Ha) s -= (T)g2 * Ha[off];
    if (Hb) s -= (T)g2 * Hb[off];
    return s;
}

// Work of one workgroup: crossbar `tile` of the batch, job `job`, output tile (I, J).
// The workgroups that invert a pivot tile at the end of the launch (output tile
// `special` = I nb + J of every job and crossbar; -1: none) come first in dispatch
// order, so that their serial inversions start with the launch instead of after
// the other updates.
// With eight jobs or more (batches), job g = tile nj + job runs on XCD g % 8:
// workgroups are dispatched round-robin over the 8 XCDs by linear index, and each
// XCD takes its jobs one after another, all of a job's workgroups together, so the
// pivot-row and pivot-column tiles that every workgroup of a job reads are fetched
// into that XCD's L2 once.  The grid then holds 8 ceil(jobs / 8) jobs' workgroups
// (gj_grid); those of the missing jobs exit at once.  A single crossbar's one or
// two jobs are spread over the whole grid instead.
struct GJSlot {
    int tile, job, I, J;
    bool valid;
};

inline dim3 gj_grid(int nj, int tiles, int batch)
{
    const int jobs = nj * batch;
    if (jobs >= 8) return dim3((unsigned)(8 * ((jobs + 7) / 8) * tiles));
    return dim3((unsigned)(nj * tiles), (unsigned)batch);
}

__device__ inline GJSlot gj_slot(int nb, int nj, int batch, int special)
{
    const int tiles = nb * nb, jobs = nj * batch;
    GJSlot s;
    s.valid = true;
    int IJ;
    if (jobs >= 8) {
        const int L = blockIdx.x, xcd = L & 7, local = L >> 3;
        const int per_xcd = (jobs + 7) / 8;
        int jl;
        if (special < 0) {
            jl = local / tiles;
            IJ = local % tiles;
        } else if (local < per_xcd) {
            jl = local;
            IJ = special;
        } else {
            const int r = local - per_xcd, per = tiles - 1;
            jl = r / per;
            const int q = r % per;
            IJ = q < special ? q : q + 1;
        }
        const int g = 8 * jl + xcd;
        s.valid = g < jobs;
        s.tile = g / nj;
        s.job = g % nj;
        s.I = IJ / nb;
        s.J = IJ % nb;
        return s;
    }
    int L = blockIdx.y * gridDim.x + blockIdx.x;
    if (special >= 0 && L < jobs) {
        s.tile = L / nj;
        s.job = L % nj;
        s.I = special / nb;
        s.J = special % nb;
        return s;
    }
    if (special >= 0) {
        L -= jobs;
        const int per = tiles - 1;
        s.tile = L / (nj * per);
        const int rem = L % (nj * per);
        s.job = rem / per;
        const int q = rem % per;
        IJ = q < special ? q : q + 1;
    } else {
        s.tile = L / (nj * tiles);
        const int rem = L % (nj * tiles);
        s.job = rem / tiles;
        IJ = rem % tiles;
    }
    s.I = IJ / nb;
    s.J = IJ % nb;
    return s;
}

// Job `j` of the launch for crossbar `tile` of a batch of one shape: the job's
// working buffers offset to that crossbar (a plan has one crossbar and keeps its own
// pointers), and in *H the crossbar's H blocks.  The job is chosen field by field
// and the arguments are never written, so that they stay in the kernel-argument
// segment: a runtime index into them, or a write, makes the compiler copy the whole
// argument block to per-lane scratch memory in every thread.
template <typename T>
__device__ inline GJJob batch_job(const GJArgs& a, int j, int tile, T** H)
{
    GJJob job;
    job.row = j ? a.job[1].row : a.job[0].row;
    job.next = j ? a.job[1].next : a.job[0].next;
    job.dep_a = j ? a.job[1].dep_a : a.job[0].dep_a;
    job.dep_b = j ? a.job[1].dep_b : a.job[0].dep_b;
    const int64_t t = tile;
    for (int k = 0; k < 2; ++k) {
        job.S[k] = reinterpret_cast<T*>(j ? a.job[1].S[k] : a.job[0].S[k]) + t * a.s_stride;
        job.P[k] = reinterpret_cast<T*>(j ? a.job[1].P[k] : a.job[0].P[k]) + t * a.p_stride;
    }
    T* W = reinterpret_cast<T*>(j ? a.job[1].W : a.job[0].W);
    job.W = W ? W + t * a.w_stride : nullptr;
    *H = reinterpret_cast<T*>(a.H) + t * a.h_stride;
    return job;
}

template <typename T>
__device__ inline const T* slot_ptr(const T* H, int n_p, int row)
{
    return row < 0 ? nullptr : H + (int64_t)row * n_p * n_p;
}

// Form the first pivot block of each job (chain start or twist) into its S[0] and
// invert its pivot tile (0,0) into its P[0].
template <typename T>
__global__ __launch_bounds__(256) void gj_form_kernel(GJArgs a, int nj)
{
    __shared__ __align__(32) T lds[kTile * kLd + 4 * kTile];
    const GJSlot sl = gj_slot(a.nb, nj, a.batch, 0);
    if (!sl.valid) return;
    T* H;
    const GJJob job = batch_job<T>(a, sl.job, sl.tile, &H);
    int* tbad = a.tile_bad ? a.tile_bad + sl.tile : nullptr;
    const int I = sl.I, J = sl.J;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const T* E = slot_ptr<T>(H, a.n_p, job.row);
    const T* Ha = slot_ptr<T>(H, a.n_p, job.dep_a);
    const T* Hb = slot_ptr<T>(H, a.n_p, job.dep_b);
    typename Frag<T>::acc_t acc[4];
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = 64 * I + out_row<T>(w, l, v), cc = 64 * J + 16 * C + (l & 15);
            acc[C][v] = form_elem<T>(E, Ha, Hb, frg<T>(rr, cc, a.n_p), a.g2, rr, cc, a.n);
        }
    store_acc<T>(acc, reinterpret_cast<T*>(job.S[0]), a.n_p, 64 * I, 64 * J, w, l);
    if (I == 0 && J == 0) {
        T* const W = reinterpret_cast<T*>(job.W);
        invert_tile<T>(acc, lds, reinterpret_cast<T*>(job.P[0]), a.flags, a.diag, min(a.n, kTile), w, l, tbad, W);
        if (W) store_acc<T>(acc, W + (int64_t)a.nb * kTile * kTile, kTile, 0, 0, w, l);   // the tile itself
    }
}

// Output tile (I, J) of pivot block k, held in acc: stored into the next working
// copy, and the pivot tile (k+1, k+1) inverted; after the last pivot block, stored as
// H_row[I][J] over E_row, then the chain's next pivot block E_next - g^2 H_row formed
// (tile (0, 0) inverted).  lds: the workgroup's operand area, free when called.
template <typename T, bool NS, bool INV = true>
__device__ inline void gj_finish_tile(typename Frag<T>::acc_t (&acc)[4], const GJArgs& a, const GJJob& job, T* H,
                                      T* Sout, T* Pout, int* tbad, int I, int J, int k, T* lds, T* lds2, int w, int l)
{
    const int nb = a.nb, n_p = a.n_p, r0 = 64 * I, c0 = 64 * J;
    T* const W = reinterpret_cast<T*>(job.W);
    if (k != nb - 1) {
        store_acc<T>(acc, Sout, n_p, r0, c0, w, l);
        if (INV && I == k + 1 && J == k + 1) {
            // a warm start exists once the chain is past its first row (the twist row
            // has two neighbours and no such inverse)
            const bool warm = job.dep_b < 0 && job.row != 0 && job.row != a.m - 1;
            invert_pivot<T, NS>(acc, lds, lds2, Pout, W ? W + (int64_t)(k + 1) * kTile * kTile : nullptr, nb, warm, a.flags,
                                a.diag, max(0, min(a.n - kTile * (k + 1), kTile)), w, l, tbad);
        }
        return;
    }
    // Last pivot block: acc holds H_row[I][J]; store it over E_row, then form the
    // chain's next pivot block E_next - g^2 H_row.  H and E are fragment-tiled, and
    // each wave holds four whole 16x16 fragment tiles of the output tile (its rows
    // 16w..16w+15), so they pass through the wave's own quarter of the LDS area:
    // every global access is then a contiguous 16 bytes per lane, where element-wise
    // accesses touch all sixteen cache lines of a fragment tile per instruction.
    lds_barrier();                       // the area is free: the product that read it is done
    T* st = lds + w * 1024;
    const int64_t tb = ((int64_t)((r0 >> 4) + w) * (n_p >> 4) + (c0 >> 4)) * 256;
    const bool form = job.next >= 0;
    T e[4][4];
    if (form) {
        const T* En = H + (int64_t)job.next * n_p * n_p + tb;
#pragma unroll
        for (int C = 0; C < 4; ++C)
#pragma unroll
            for (int t = 0; t < 4; ++t) e[C][t] = En[C * 256 + frg_slot<T>(l, t)];
    }
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) st[C * 256 + frg<T>(Frag<T>::drow(l >> 4, v), l & 15, 16)] = acc[C][v];
    wave_lds_sync();
    T* Hr = H + (int64_t)job.row * n_p * n_p + tb;
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int t = 0; t < 4; ++t) Hr[C * 256 + frg_slot<T>(l, t)] = st[C * 256 + frg_slot<T>(l, t)];
    if (!form) return;
    wave_lds_sync();
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int t = 0; t < 4; ++t) st[C * 256 + frg_slot<T>(l, t)] = e[C][t];
    wave_lds_sync();
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = r0 + out_row<T>(w, l, v), cc = c0 + 16 * C + (l & 15);
            const T ev = st[C * 256 + frg<T>(Frag<T>::drow(l >> 4, v), l & 15, 16)];
            acc[C][v] = (rr < a.n && cc < a.n) ? ev - (T)a.g2 * acc[C][v] : (T)(rr == cc ? 1 : 0);
        }
    store_acc<T>(acc, Sout, n_p, r0, c0, w, l);
    // tile 0 of the next row's pivot block, from this row's inverse of its tile 0
    if (INV && I == 0 && J == 0)
        invert_pivot<T, NS>(acc, lds, lds2, Pout, W, nb, true, a.flags, a.diag, min(a.n, kTile), w, l, tbad);
}

// Pivot block k of the current row of every job; parity = (step*nb + k) & 1.
template <typename T, bool NS>
__global__ __launch_bounds__(256, NS ? 2 : 3) void gj_step_kernel(GJArgs a, int nj, int step, int k)
{
    // B operands (the A operands go from memory straight into registers), also the
    // area of the pivot-tile inversion and of the staged output tiles; the
    // Newton-Schulz round (NS) needs a second area.
    __shared__ __align__(32) T sB[kTile * kLd + 4 * kTile];
    __shared__ __align__(32) T sA[NS ? kTile * kLd + 4 * kTile : 1];
    T* const area = NS ? sA : sB;
    const int nb = a.nb, n_p = a.n_p;
    // the pivot tile this launch's inverting workgroups own: (k+1, k+1), or (0, 0) of
    // the next row's pivot block after the last pivot of a row
    const int special = k != nb - 1 ? (k + 1) * nb + (k + 1) : (a.job[0].next >= 0 || (nj > 1 && a.job[1].next >= 0)) ? 0 : -1;
    const GJSlot sl = gj_slot(nb, nj, a.batch, special);
    if (!sl.valid) return;
    T* H;
    const GJJob job = batch_job<T>(a, sl.job, sl.tile, &H);
    int* tbad = a.tile_bad ? a.tile_bad + sl.tile : nullptr;
    const int I = sl.I, J = sl.J;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int par = (int)(((int64_t)step * nb + k) & 1);
    // (selects, not a runtime index, which would put the pointer pairs in scratch)
    const T* Sin = reinterpret_cast<const T*>(par ? job.S[1] : job.S[0]);
    T* Sout = reinterpret_cast<T*>(par ? job.S[0] : job.S[1]);
    const T* Pin = reinterpret_cast<const T*>(par ? job.P[1] : job.P[0]);
    T* Pout = reinterpret_cast<T*>(par ? job.P[0] : job.P[1]);
    using acc_t = typename Frag<T>::acc_t;
    acc_t acc[4];
#pragma unroll
    for (int C = 0; C < 4; ++C) acc[C] = acc_t{0, 0, 0, 0};

    const int r0 = 64 * I, c0 = 64 * J, pk = 64 * k;
    T av[4][4], vb[kPer];
    if (I != k && J != k) {
        T a2[4][4];
        fetch_afrag<T>(av, Pin, kTile, 0, 0, w, l);
        fetch_tile<T>(vb, Sin, n_p, pk, c0);
        fetch_afrag<T>(a2, Sin, n_p, r0, pk, w, l);
        load_acc<T>(acc, Sin, n_p, r0, c0, w, l);
        put_B<T>(sB, vb);
        __syncthreads();
        acc_t x[4];
#pragma unroll
        for (int C = 0; C < 4; ++C) x[C] = acc_t{0, 0, 0, 0};
        tile_mma_r<T>(x, av, (T)1, sB, w, l);           // X = P^{-1} S[k][J]
        __syncthreads();
#pragma unroll
        for (int C = 0; C < 4; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) {               // X becomes the next B operand
                const int kk = out_row<T>(w, l, v);
                sB[(16 * C + (l & 15)) * kLd + (kk & ~15) + Frag<T>::slot(kk & 15)] = x[C][v];
            }
        __syncthreads();
        tile_mma_r<T>(acc, a2, (T)-1, sB, w, l);        // S[I][J] - S[I][k] X
    } else if (I == k && J != k) {
        fetch_afrag<T>(av, Pin, kTile, 0, 0, w, l);
        fetch_tile<T>(vb, Sin, n_p, pk, c0);
        put_B<T>(sB, vb);
        __syncthreads();
        tile_mma_r<T>(acc, av, (T)1, sB, w, l);         // P^{-1} S[k][J]
    } else if (I != k && J == k) {
        fetch_afrag<T>(av, Sin, n_p, r0, pk, w, l);
        fetch_tile<T>(vb, Pin, kTile, 0, 0);
        put_B<T>(sB, vb);
        __syncthreads();
        tile_mma_r<T>(acc, av, (T)-1, sB, w, l);        // -S[I][k] P^{-1}
    } else {
        load_acc<T>(acc, Pin, kTile, 0, 0, w, l);       // P^{-1}
    }

    gj_finish_tile<T, NS>(acc, a, job, H, Sout, Pout, tbad, I, J, k, area, sB, w, l);
}

// Column workgroups of a batch (eight jobs or more, nb >= 3): one workgroup per
// column block J of every job, job g on XCD g % 8 as in gj_slot, the column that
// holds the tile inverted at the end (`scol`, -1: none) first in dispatch order.
__device__ inline GJSlot gj_col_slot(int nb, int nj, int batch, int scol)
{
    const int jobs = nj * batch;
    const int L = blockIdx.x, xcd = L & 7, local = L >> 3;
    const int per_xcd = (jobs + 7) / 8;
    int jl, J;
    if (scol < 0) {
        jl = local / nb;
        J = local % nb;
    } else if (local < per_xcd) {
        jl = local;
        J = scol;
    } else {
        const int r = local - per_xcd, per = nb - 1;
        jl = r / per;
        const int q = r % per;
        J = q < scol ? q : q + 1;
    }
    const int g = 8 * jl + xcd;
    GJSlot s;
    s.valid = g < jobs;
    s.tile = g / nj;
    s.job = g % nj;
    s.I = 0;
    s.J = J;
    return s;
}

inline dim3 gj_col_grid(int nj, int nb, int batch)
{
    return dim3((unsigned)(8 * ((nj * batch + 7) / 8) * nb));
}

// Pivot block k of the current row of every job, one column block J per workgroup:
// X = P^{-1} S[k][J] (P^{-1} itself for J = k) is formed once and becomes tile (k, J);
// every other tile of the column is S[I][J] - S[I][k] X (-S[I][k] P^{-1} for J = k).
// The same products as gj_step_kernel's, in the same order, so the same bits; the
// column's three other workgroups there each form X again.  The tile to invert at
// the end of the launch is the column's last.
template <typename T, bool NS>
__global__ __launch_bounds__(256, 2) void gj_col_kernel(GJArgs a, int nj, int step, int k)
{
    __shared__ __align__(32) T sA[kTile * kLd + 4 * kTile];
    __shared__ __align__(32) T sB[kTile * kLd];
    const int nb = a.nb, n_p = a.n_p;
    const bool last = k == nb - 1;
    const int scol = !last ? k + 1 : (a.job[0].next >= 0 || (nj > 1 && a.job[1].next >= 0)) ? 0 : -1;
    const GJSlot sl = gj_col_slot(nb, nj, a.batch, scol);
    if (!sl.valid) return;
    T* H;
    const GJJob job = batch_job<T>(a, sl.job, sl.tile, &H);
    int* tbad = a.tile_bad ? a.tile_bad + sl.tile : nullptr;
    const int J = sl.J;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int par = (int)(((int64_t)step * nb + k) & 1);
    const T* Sin = reinterpret_cast<const T*>(par ? job.S[1] : job.S[0]);
    T* Sout = reinterpret_cast<T*>(par ? job.S[0] : job.S[1]);
    const T* Pin = reinterpret_cast<const T*>(par ? job.P[1] : job.P[0]);
    T* Pout = reinterpret_cast<T*>(par ? job.P[0] : job.P[1]);
    using acc_t = typename Frag<T>::acc_t;
    const int c0 = 64 * J, pk = 64 * k;
    // the row of this column whose tile is inverted at the end (-1: none)
    const int srow = J == scol ? (last ? 0 : k + 1) : -1;

    // the rows other than k in increasing order, the inverted tile's row last
    const int s1 = srow < 0 ? k : min(k, srow), s2 = srow < 0 ? nb : max(k, srow);
    const int rows = nb - 1;
    auto row_at = [&](int t) {
        if (srow >= 0 && t == rows - 1) return srow;
        int I = t;
        if (I >= s1) ++I;
        if (I >= s2) ++I;
        return I;
    };
    // operands of a row's update: S[I][k], and S[I][J] (0 for J = k)
    auto fetch_row = [&](int I, T (&v)[kPer], acc_t (&acc)[4]) {
        fetch_tile<T>(v, Sin, n_p, 64 * I, pk);
        if (J != k) {
            load_acc<T>(acc, Sin, n_p, 64 * I, c0, w, l);
        } else {
#pragma unroll
            for (int C = 0; C < 4; ++C) acc[C] = acc_t{0, 0, 0, 0};
        }
    };
    // The barriers order LDS only: no thread reads another's global writes within the
    // launch.
    acc_t x[4];
    if (J != k) {
        T v0[kPer], v1[kPer];
        fetch_tile<T>(v0, Pin, kTile, 0, 0);
        fetch_tile<T>(v1, Sin, n_p, pk, c0);
        put_A<T>(sA, v0, (T)1);
        put_B<T>(sB, v1);
        lds_barrier();
#pragma unroll
        for (int C = 0; C < 4; ++C) x[C] = acc_t{0, 0, 0, 0};
        tile_mma<T>(x, sA, sB, w, l);                   // X = P^{-1} S[k][J]
        lds_barrier();
    } else {
        load_acc<T>(x, Pin, kTile, 0, 0, w, l);         // X = P^{-1}
    }
#pragma unroll
    for (int C = 0; C < 4; ++C)
#pragma unroll
        for (int v = 0; v < 4; ++v) {                   // X becomes the B operand of the column
            const int kk = out_row<T>(w, l, v);
            sB[(16 * C + (l & 15)) * kLd + (kk & ~15) + Frag<T>::slot(kk & 15)] = x[C][v];
        }
    gj_finish_tile<T, NS, false>(x, a, job, H, Sout, Pout, tbad, k, J, k, sA, sB, w, l);   // row k: never inverted

    // the other rows, the inverted tile's row after them
    auto update = [&](int I, acc_t (&ac)[4]) {
        T vc[kPer];
        fetch_row(I, vc, ac);
        lds_barrier();                                   // sA free, X in sB visible
        put_A<T>(sA, vc, (T)-1);
        lds_barrier();
        tile_mma<T>(ac, sA, sB, w, l);                   // S[I][J] - S[I][k] X
    };
    const int plain = srow >= 0 ? rows - 1 : rows;
    for (int t = 0; t < plain; ++t) {
        const int I = row_at(t);
        acc_t ac[4];
        update(I, ac);
        gj_finish_tile<T, NS, false>(ac, a, job, H, Sout, Pout, tbad, I, J, k, sA, sB, w, l);
    }
    if (srow >= 0) {
        acc_t ac[4];
        update(srow, ac);
        gj_finish_tile<T, NS>(ac, a, job, H, Sout, Pout, tbad, srow, J, k, sA, sB, w, l);
    }
}


// One pivot-block launch: column or tile workgroups, with the Newton-Schulz pivot tiles
// when the jobs carry warm-start slots.
template <typename T>
void launch_step(const GJArgs& f, int nj, int st, int k, bool cols, hipStream_t s)
{
    const int nb = f.nb, tiles = nb * nb;
    const bool ns = f.job[0].W != nullptr;
    if (cols && ns)
        hipLaunchKernelGGL((gj_col_kernel<T, true>), gj_col_grid(nj, nb, f.batch), dim3(256), 0, s, f, nj, st, k);
    else if (cols)
        hipLaunchKernelGGL((gj_col_kernel<T, false>), gj_col_grid(nj, nb, f.batch), dim3(256), 0, s, f, nj, st, k);
    else if (ns)
        hipLaunchKernelGGL((gj_step_kernel<T, true>), gj_grid(nj, tiles, f.batch), dim3(256), 0, s, f, nj, st, k);
    else
        hipLaunchKernelGGL((gj_step_kernel<T, false>), gj_grid(nj, tiles, f.batch), dim3(256), 0, s, f, nj, st, k);
}

template <typename T>
hipError_t launch_factor(GJArgs a, hipStream_t s)
{
    const int m = a.m, kt = m / 2, nb = a.nb, tiles = nb * nb;
    const int top_len = kt, bot_len = m - 1 - kt;
    GJJob top = a.job[0], bot = a.job[1];    // buffers provided by the caller
    hipError_t e;
    // chain starts: S_0 = E_0 (top), S'_{m-1} = E_{m-1} (bottom)
    {
        GJArgs f = a;
        int nj = 0;
        if (top_len > 0) { f.job[nj] = top; f.job[nj].row = 0; f.job[nj].dep_a = f.job[nj].dep_b = -1; ++nj; }
        if (bot_len > 0) { f.job[nj] = bot; f.job[nj].row = m - 1; f.job[nj].dep_a = f.job[nj].dep_b = -1; ++nj; }
        if (nj > 0) {
            hipLaunchKernelGGL(gj_form_kernel<T>, gj_grid(nj, tiles, a.batch), dim3(256), 0, s, f, nj);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    const int steps = top_len > bot_len ? top_len : bot_len;
    for (int st = 0; st < steps; ++st) {
        GJArgs f = a;
        int nj = 0;
        if (st < top_len) {
            f.job[nj] = top;
            f.job[nj].row = st;
            f.job[nj].next = (st + 1 < kt) ? st + 1 : -1;
            ++nj;
        }
        if (st < bot_len) {
            f.job[nj] = bot;
            f.job[nj].row = m - 1 - st;
            f.job[nj].next = (m - 2 - st > kt) ? m - 2 - st : -1;
            ++nj;
        }
        const bool cols = nj * a.batch >= 8 && nb >= 3;
        for (int k = 0; k < nb; ++k) {
            launch_step<T>(f, nj, st, k, cols, s);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    // twist block K = E_kt - g^2 (H_{kt-1} + H'_{kt+1})
    GJArgs f = a;
    f.job[0] = top;
    f.job[0].row = kt;
    f.job[0].dep_a = (kt >= 1) ? kt - 1 : -1;
    f.job[0].dep_b = (kt + 1 <= m - 1) ? kt + 1 : -1;
    f.job[0].next = -1;
    hipLaunchKernelGGL(gj_form_kernel<T>, gj_grid(1, tiles, a.batch), dim3(256), 0, s, f, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int k = 0; k < nb; ++k) {
        launch_step<T>(f, 1, 0, k, a.batch >= 8 && nb >= 3, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace xbk

hipError_t xbk_launch_factor(const xbk::GJArgs& a, bool fp32, hipStream_t s)
{
    return fp32 ? xbk::launch_factor<float>(a, s) : xbk::launch_factor<double>(a, s);
}

// Shared device definitions for the gfx950 crossbar solver kernels.
//
// Matrix-core fragments (wave64, 16x16 output tile):
//   v_mfma_f64_16x16x4f64 : A lane l = A[l%16][l/16], B lane l = B[l/16][l%16],
//                           D lane l item v = D[l/16 + 4v][l%16]
//   v_mfma_f32_16x16x4f32 : A, B as above,  D lane l item v = D[4(l/16) + v][l%16]
// (measured on gfx950 with a one-hot probe).
//
// The contraction index K is processed in chunks of 16.  Within a chunk,
// MFMA step t of lane-group q = l/16 uses k = kidx(q, t), chosen so that
// the four k values a lane touches are exactly the four output rows the
// same lane holds in the D layout:
//   f64: kidx(q, t) = q + 4t     f32: kidx(q, t) = 4q + t
// A row-major matrix whose columns are permuted inside each 16-chunk by
// slot(k) = position of k in (q, t) order makes every lane's four A values
// contiguous (one 32-byte or 16-byte load).  This "chunk-permuted row-major"
// (CPR) layout is used for the Gauss-Jordan working blocks and for the
// panels of right-hand sides, stored [column][slot(k)].
//
// Blocks that stream through the matrix cores (E_i, then H_i, and the
// Newton-Schulz iterates) use a fragment-tiled (FRG) layout instead: 16x16
// tiles in row-major tile order, each tile stored in A-operand lane order, so
// that a wave reads one tile with fully contiguous 16-byte loads (1 KB per
// load instruction) rather than 16 short row segments:
//   f64: lane l = 16q + r holds (r, kidx(q, t)), t = 0..3, at 128 (t >> 1) + 2 l + (t & 1)
//   f32: lane l holds (r, kidx(q, t)) at 4 l + t
// The same slots hold the D tile of an MFMA transposed: with the A slot fed
// from tile rows of B and the B slot from tile rows of A, lane l item v of D
// is element (r, kidx(q, v)) of the matching tile of A B^T, stored in place.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

namespace xbk {

constexpr int kWave = 64;
constexpr int kTile = 64;          // block-inversion tile edge (rows/cols)
constexpr int kSlabCols = 16;      // input vectors per workgroup in the sweeps

template <typename T> struct Frag;
template <> struct Frag<double> {
    using acc_t = d4_t;
    // k (0..15) of MFMA step t for lane group q
    __host__ __device__ static constexpr int kidx(int q, int t) { return q + 4 * t; }
    // slot of k inside its 16-chunk in CPR order (inverse of kidx)
    __host__ __device__ static constexpr int slot(int k) { return 4 * (k & 3) + (k >> 2); }
    // row (within the 16-row tile) of output item v for lane group q
    __host__ __device__ static constexpr int drow(int q, int v) { return q + 4 * v; }
    __device__ static inline acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Frag<float> {
    using acc_t = f4_t;
    __host__ __device__ static constexpr int kidx(int q, int t) { return 4 * q + t; }
    __host__ __device__ static constexpr int slot(int k) { return k; }
    __host__ __device__ static constexpr int drow(int q, int v) { return 4 * q + v; }
    __device__ static inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// CPR offset of (r, k) in a row-major matrix with leading dimension ld.
template <typename T>
__host__ __device__ inline int64_t cpr(int64_t r, int k, int ld) {
    return r * ld + (k & ~15) + Frag<T>::slot(k & 15);
}

// FRG slot of item t of lane l inside a 256-element tile.
template <typename T>
__host__ __device__ constexpr int frg_slot(int l, int t) {
    return sizeof(T) == 8 ? 128 * (t >> 1) + 2 * l + (t & 1) : 4 * l + t;
}

// FRG offset of (r, c) in an n_p x n_p block.
template <typename T>
__host__ __device__ inline int64_t frg(int r, int c, int n_p) {
    const int k = c & 15;
    const int q = sizeof(T) == 8 ? (k & 3) : (k >> 2);     // inverse of kidx
    const int t = sizeof(T) == 8 ? (k >> 2) : (k & 3);
    const int64_t tile = (int64_t)(r >> 4) * (n_p >> 4) + (c >> 4);
    return tile * 256 + frg_slot<T>(16 * q + (r & 15), t);
}

// (row, column) held at FRG offset e of an n_p x n_p block.
template <typename T>
__host__ __device__ inline void frg_rc(int64_t e, int n_p, int& r, int& c) {
    const int64_t tile = e >> 8;
    const int s = (int)(e & 255);
    int l, t;
    if (sizeof(T) == 8) {
        l = (s & 127) >> 1;
        t = 2 * (s >> 7) + (s & 1);
    } else {
        l = s >> 2;
        t = s & 3;
    }
    const int kt = n_p >> 4;
    r = 16 * (int)(tile / kt) + (l & 15);
    c = 16 * (int)(tile % kt) + Frag<T>::kidx(l >> 4, t);
}

// Maximum that keeps NaN: fmax drops a NaN as soon as a number follows it, which
// would let a non-finite correction or estimate pass a convergence or routing test.
__device__ __forceinline__ double nan_max(double a, double b)
{
    return (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
}

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store of the wave; kernels whose threads
// never read each other's global writes within a launch use this instead, so
// that stores (node voltages, forward-sweep panels) drain while the next
// row's products run.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Device error flags (sticky, cleared by assemble).  kNsFail is internal: a
// Newton-Schulz inverse that missed its tolerance (the factor then reruns
// with Gauss-Jordan elimination).
// kNsUsed + c: launches Newton-Schulz schedule c needed in the last asynchronous
// factorization (0 if it did not finish within its budget).
enum : int { kErrInput = 0, kErrPivot = 1, kErrConv = 2, kIrIters = 3, kNsFail = 4, kNsUsed = 5,
             kNumFlags = 8 };

// Plan diagnostics (64-bit words, reset by assembly and, for the backward error,
// by each solve that measures it): the smallest pivot the factor met, as an
// order-preserving key (pivot_key), and the bit pattern of the largest normwise
// backward error of a solved batch (a non-negative double, so its bits order
// like its value; NaN above everything).
enum : int { kDiagMinPivot = 0, kDiagBackErr = 1, kNumDiag = 4 };

// Key whose unsigned order is the order of the doubles (NaN below everything).
__host__ __device__ inline unsigned long long pivot_key(double x)
{
    if (x != x) return 0ull;
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
constexpr unsigned long long kPivotKeyInf = 0xFFF0000000000000ull;   // pivot_key(+inf)

// Fold a wave's candidate pivots (+inf where a lane has none) into the plan's
// smallest pivot; a pivot that is not positive (or NaN) raises kErrPivot.
__device__ inline void record_min_pivot(double v, unsigned long long* diag, int* flags);

constexpr int kNsMaxIter = 6;      // Newton-Schulz steps allowed per chain row
constexpr int kNsMaxIterTwist = 10;

// Newton-Schulz inversion of the pivot blocks: per chain, the formed pivot
// block S, two iterates X, the residual Q = I - X S, its transpose and its square.
struct NSChain {
    void* S;
    void* X[2];
    void* Q;
    double* dprev;       // [2][n_p] diagonal of the pivot block of chain row i at [i & 1]
};

struct NSJob {
    int row, dep_a, dep_b;   // pivot block E_row - g^2 (H_dep_a + H_dep_b)
    int warm;                // 1: start from H_dep_a corrected on the diagonal; 0: from diag(S)^{-1}
    int chain;               // which NSChain buffers
};

// Device-driven schedules of the Newton-Schulz factor (top chain, bottom chain,
// twist).  Each launch ("slot") of a schedule reads its state, does its phase
// (form the pivot block and the first iterate, or one of the launches of a round
// or step) and writes the next state into the other parity, so no
// launch is spent on a row that has already converged.
enum : int { kNsForm = 0, kNsResid = 1, kNsQx = 2, kNsUpdate = 3, kNsFinished = 4 };
struct NSState {
    int row;      // crossbar row being inverted
    int phase;    // kNs*
    int it;       // Newton-Schulz step of the row
    int xb;       // which of the chain's two X buffers holds the current iterate
    int slots;    // slot count at which the schedule finished (kNsFinished), else 0
};

__device__ inline void record_min_pivot(double v, unsigned long long* diag, int* flags)
{
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off);
        v = (o < v || o != o) ? o : v;
    }
    if ((threadIdx.x & 63) == 0 && !(v == __builtin_inf())) {
        if (!(v > 0.0)) atomicOr(flags + kErrPivot, 1);
        atomicMin(diag + kDiagMinPivot, pivot_key(v));
    }
}

struct NSArgs {
    int m, n, n_p;
    double g2;
    void* H;                 // [m][n_p][n_p] FRG: E_i on entry, H_i on exit
    NSChain ch[2];           // buffers of the top chain (and the twist row), bottom chain
    NSState* state;          // [2 parities][3 schedules: top chain, bottom chain, twist]
    double* part;            // [2 chains][(n_p/32)^2] per-workgroup max |I - X P| of the current step
    int* flags;
    unsigned long long* diag;   // [kNumDiag] plan diagnostics
    int max_iter;
};

// Crossbar blockIdx.y of a batch of one shape reads G + y m n and writes E, c, fr,
// ip, q and Gc at y times one crossbar's size (gridDim.y = 1 for a plan).
struct CondenseArgs {
    const double* G;     // [m][n] user conductances
    int m, n, n_p;
    double g_wl, g_bl, g_src, g_sense;
    void* E;             // [m][n_p][n_p] FRG, element type of the factor
    double* c;           // [m][n_p]  condensed source coupling c_i
    double* fr;          // [m][n]    g_wl / p_{j-1} (0 at j = 0): forward Thomas ratios of T_i
    double* ip;          // [m][n]    1 / p_j
    double* q;           // [m][n]    bit-line self conductance q_ij
    double* Gc;          // [m][n]    copy of G
    int* flags;
    int* tile_bad = nullptr;   // batches: per-crossbar flag, set for a bad conductance
};

// One inversion in flight: the pivot block of crossbar row `row`.
struct GJJob {
    int row;             // row whose pivot block is being inverted
    int next;            // row whose pivot block this one feeds (-1: none)
    int dep_a, dep_b;    // rows whose inverses enter the pivot block (-1: none)
    void* S[2];          // working copies of the pivot block, [n_p][n_p] CPR each
    void* P[2];          // inverted 64x64 pivot tiles, CPR each
    void* W = nullptr;   // batches: [2][nb][64][64] CPR, the chain's last inverse of each pivot
                         // tile and the tile itself (warm starts of the next row's inverses),
                         // or null (elimination only)
};

struct GJArgs {
    int m, n, n_p, nb;   // nb = n_p / 64 tile rows per block
    double g2;           // g_bl^2: coupling of neighbouring row blocks
    void* H;             // [m][n_p][n_p] FRG: E_i on entry, pivot inverse H_i on exit
    GJJob job[2];        // top and bottom chains (one job for the twist row)
    int* flags;
    unsigned long long* diag;   // [kNumDiag] plan diagnostics
    // batched crossbars of one shape (blockIdx.y): crossbar t uses H + t * h_stride and the
    // jobs' S and P buffers + t * s_stride, t * p_stride (elements); batch = 1 for a plan
    int batch = 1;
    int64_t h_stride = 0, s_stride = 0, p_stride = 0, w_stride = 0;
    int* tile_bad = nullptr;   // batches: per-crossbar flag, set for a pivot that is not positive
};

struct SweepArgs {
    int m, n, n_p, B, nslab;
    double g_bl, g_sense;
    const void* H;       // [m][n_p][n_p] FRG block inverses H_i
    const double* c;     // [m][n_p]
    const double* V;     // [B][m] user inputs
    void* Z;             // [nslab][m][16][n_p]: forward sweep z_i (or the correction d_i)
    double* Iout;        // [B][n]
    // word-line recovery fused into the float64 back sweep (node_v == nullptr: skipped)
    double* node_v;      // [B][2mn]
    double* sink;        // [128] target of the L2 pulls' keep-alive store (taken only by chance)
    const double* Gc;    // [m][n]
    const double* fr;    // [m][n]
    const double* ip;    // [m][n]
    double g_src, g_wl;
    // iterative refinement (float sweeps): correction of the float64 solution U
    int iter;            // 0: right-hand side V c; > 0: right-hand side R
    int max_iter;        // sweeps allowed in total
    double tol;
    const void* R;       // [nslab][m][16][n_p] float residual panels (iter > 0)
    const double* Uin;   // [nslab][m][16][n_p] solution before this sweep (iter > 0)
    double* Uout;        // solution after it
    double* dnorm;       // [nslab][16] largest correction of the previous sweep, per vector
    int* slab_done;      // [nslab]
    int* slab_final;     // [nslab] which U buffer holds the final solution
    int* flags;
    // tol < 0: the sweep only applies the factor (Uout = Uin + M^-1 R); it keeps no
    // convergence state (dnorm, slab_done, slab_final and flags are not written)
    // batched crossbars of one shape (float64, currents only): `batch` crossbars of
    // `slabs_per` slabs each, crossbar t's H, c, V, Z and Iout at t times the size of one
    // crossbar's; workgroups are mapped so that a crossbar's slabs share an XCD (and its
    // L2).  batch = 1 for a plan.  `slab` is set per workgroup inside the kernel.
    int batch = 1, slabs_per = 0;
    int slab = 0;
    const int* tile_bad = nullptr;   // batches: crossbars flagged bad get NaN currents
    int unit = 0;                    // 1: input vector b is the unit vector e_b (V is not read)
    // 1: reciprocal ordering (a plan of an m' x n' crossbar with n' > m', solved as its
    // n' x m' reciprocal): the inputs V [B][n] drive the bit-line terminations of row
    // m-1, so the right-hand side is g_sense V[b][n-1-k] at row m-1 and zero elsewhere,
    // and the word lines have no sources
    int term = 0;
};

struct ResidualArgs {
    int m, n, n_p, B, nslab;
    double g_bl, g_wl;
    const double* V;     // [B][m]
    const double* c;     // [m][n_p]
    const double* fr;
    const double* ip;
    const double* q;
    const double* Gc;
    const double* U;     // [nslab][m][16][n_p] current solution (float positions)
    void* R;             // [nslab][m][16][n_p] float residual
    const int* slab_done;
    // Krylov refinement: Rd != nullptr writes the float64 result there instead of the
    // float R; matvec = 1 writes the product A u of the condensed matrix (V not read)
    // instead of the residual V c - A u
    double* Rd = nullptr;
    int matvec = 0;
    int term = 0;        // reciprocal ordering (see SweepArgs::term); V is [B][n]
    double g_sense = 0.0;
};

// Krylov refinement (gmres.hip): restart length and the panel geometry its batched
// vector kernels share.  A panel holds P = nslab m 16 n_p float64 values; reductions
// run over nchunk chunks of rows_per_chunk rows.
constexpr int kGmRestart = 8;              // XBAR_GMRES_RESTART
struct GmPanel {
    int m, n_p, nslab, nchunk, rows_per_chunk;
    int64_t P;
    int* slab_done;      // [nslab] converged slabs (skipped by every kernel)
    int* slab_final;     // [nslab] set to 0 (the solution buffer) when a slab stops
};

struct RecoverArgs {
    int m, n, n_p, B, nslab;
    double g_src;
    const double* V;     // [B][m]
    const double* U[2];  // float64 solutions of the refinement, U[slab_final[slab]] is final
    const int* slab_final;
    const double* fr;
    const double* ip;
    const double* Gc;
    double g_wl;
    double* node_v;      // [B][2mn]
    int term = 0;        // reciprocal ordering: no word-line sources
};

// Normwise backward error of node voltages (diagnostics.hip).
struct BackErrArgs {
    int m, n, B;
    double g_wl, g_bl, g_src, g_sense;
    const double* G;          // [m][n]
    const double* V;          // [B][m]
    const double* node_v;     // [B][2mn], paper order
    unsigned long long* diag; // [kNumDiag]: kDiagBackErr receives the batch maximum
    int rev = 0;              // G is the reciprocal crossbar's [n][m]: G[i][j] at (n-1-j) m + m-1-i
};

}  // namespace xbk

// Host-side launchers (defined in the .hip files, called by the C ABI layer).
hipError_t xbk_launch_condense(const xbk::CondenseArgs& a, bool fp32, hipStream_t s, int batch = 1);
hipError_t xbk_launch_factor(const xbk::GJArgs& a, bool fp32, hipStream_t s);
hipError_t xbk_launch_ns_init(const xbk::NSArgs& a, hipStream_t s);
hipError_t xbk_launch_ns_slots(const xbk::NSArgs& a, bool fp32, int chain, int first, int count, hipStream_t s);
hipError_t xbk_launch_ns_finish(const xbk::NSArgs& a, int launched0, int launched1, int launched2, hipStream_t s);
hipError_t xbk_launch_sweep(const xbk::SweepArgs& a, hipStream_t s);
hipError_t xbk_launch_recover(const xbk::RecoverArgs& a, hipStream_t s);
hipError_t xbk_launch_sweep_ir(const xbk::SweepArgs& a, hipStream_t s);
hipError_t xbk_launch_residual(const xbk::ResidualArgs& a, hipStream_t s);
int xbk_backward_error_max_n();     // widest crossbar the backward-error kernel measures
// Krylov refinement kernels (gmres.hip); X_i = X + i P
hipError_t xbk_gm_dots(const xbk::GmPanel& g, const double* X, int nv, const double* w, double* part, double* out,
                       int ld_out, bool add, bool sqrt_out, hipStream_t s);
hipError_t xbk_gm_axpy(const xbk::GmPanel& g, const double* X, int nv, const double* coef, int ld_coef, double* w,
                       hipStream_t s);
hipError_t xbk_gm_scale(const xbk::GmPanel& g, const double* w, const double* sc, double* v, float* Rf,
                        hipStream_t s);
hipError_t xbk_gm_lsq(const xbk::GmPanel& g, const double* Hs, const double* beta, double* y, hipStream_t s);
hipError_t xbk_gm_update(const xbk::GmPanel& g, const double* Z, const double* y, double* u, double* part, int B,
                         double tol, int it, bool last, int* flags, hipStream_t s);
hipError_t xbk_gm_currents(const xbk::GmPanel& g, int B, int n, double g_sense, const double* u, double* Iout,
                           hipStream_t s);
hipError_t xbk_gm_fill(double* x, int64_t count, double v, hipStream_t s);
hipError_t xbk_gm_add(const xbk::GmPanel& g, int nv, const double* src, int ld_src, double* dst, int ld_dst,
                      hipStream_t s);
hipError_t xbk_launch_backward_error(const xbk::BackErrArgs& a, hipStream_t s);
hipError_t xbk_launch_shift_diag(void* E, bool fp32, int m, int n, int n_p, double shift, hipStream_t s);
hipError_t xbk_launch_reset_diag(unsigned long long* diag, int which, hipStream_t s);

// Heterogeneous batches of crossbars (the partitioned crossbars of Sec. III.C at
// scale): classes of crossbars of one shape each, all of them solved by one call
// that forks the classes over a few streams and joins them back, so that the whole
// batch can be captured into one HIP graph.
//
// Two ways to solve a class (chosen per class by the caller, e.g. from the tuner's
// cache):
//  - one workgroup per crossbar (n <= 64), the whole solve in one launch
//    (tiles.hip), optionally with a crossbar's input vectors split over 2-4
//    workgroups;
//  - the plan path's kernels batched over the class (any n <= XBAR_MAX_N):
//    condensation of every row of every crossbar (one launch), the twisted block
//    Gauss-Jordan factorization of every crossbar (launches per pivot tile, each
//    covering the whole class), and the float64 currents-only sweep of every
//    crossbar's 16-vector slabs (one launch; a crossbar's slabs share an XCD).
// A class may also be solved through its reciprocal problem (`transpose`), which
// orders the row blocks by the smaller side when m < n.  The network is reciprocal:
// the current T[i][j] into the sense resistor of bit line j per volt on word line i
// equals the current into the source resistor of word line i per volt applied at the
// sense terminal of bit line j.  That is the output of the crossbar rotated by a half
// turn and transposed (its rows are the bit lines n-1..0, its columns the word lines
// m-1..0, word-line and bit-line segment resistances swapped, r_sense as its source
// resistance and r_src as its sense resistance), driven by n unit inputs.  Its row
// blocks have m unknowns instead of n, and then I = V T is one small product per
// crossbar.
// Crossbars are independent, so a bad conductance or pivot spoils only its own
// crossbar's currents (NaN).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "tiles.h"
#include "xbar.h"

namespace {

// What the kernels solve for a class: the class itself, or (transpose) its
// reciprocal problem, mi = n rows of ni = m columns with Bi = n unit inputs.
struct Inner {
    int mi, ni, Bi;
    bool unit;
    double g_wl, g_bl, g_src, g_sense;
};

struct PipeBuffers {
    void* H = nullptr;           // [T][m][n_p][n_p] FRG: E_i, then H_i
    double* c = nullptr;         // [T][m][n_p]
    double* fr = nullptr;        // [T][m][n] (condensation's Thomas ratios; unused by the currents)
    double* ip = nullptr;
    double* q = nullptr;
    double* Gc = nullptr;
    void* S[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [chain][parity][T][n_p][n_p]
    void* P[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [chain][parity][T][64][64]
    void* W[2] = {nullptr, nullptr};   // [chain][T][2][nb][64][64] last inverse of each pivot tile, the tile
    void* Z = nullptr;           // [T][slabs][m][16][n_p] forward results
    int* flags = nullptr;        // [kNumFlags]
    unsigned long long* diag = nullptr;
    double* sink = nullptr;      // [128]
    int* bad = nullptr;          // [T] crossbars with a bad conductance or pivot
    int n_p = 0, nb = 0, slabs = 0;
    double* Gt = nullptr;        // transpose: [T][n][m] the reciprocal problems' conductances
    double* Tt = nullptr;        // transpose: [T][n][m] their currents, T[i][j] = Tt[n-1-j][m-1-i]
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

constexpr int64_t kNsPivotJobs = 512;    // largest batch (jobs per launch) with warm-started pivot tiles

// Gt[t][j'][i'] = G[t][m-1-i'][n-1-j']: the crossbar turned by a half turn and transposed
__global__ void rotate_transpose_kernel(const double* __restrict__ G, double* __restrict__ Gt, int T, int m, int n)
{
    const int64_t total = (int64_t)T * m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / ((int64_t)m * n);
        const int r = (int)(e - t * m * n);
        const int jp = r / m, ip = r % m;
        Gt[e] = G[(t * m + (m - 1 - ip)) * n + (n - 1 - jp)];
    }
}

// I[t][b][j] = sum_i V[t][b][i] T[i][j] with T[i][j] = Tt[t][n-1-j][m-1-i]: 64 columns x 4
// input vectors per workgroup, the vectors' rows of V staged in LDS.
__global__ __launch_bounds__(256) void apply_reciprocal_kernel(const double* __restrict__ V,
                                                               const double* __restrict__ Tt,
                                                               double* __restrict__ I, int m, int n, int B)
{
    extern __shared__ double vs[];                       // [4][m]
    const int t = blockIdx.z, b0 = 4 * blockIdx.y, j = 64 * blockIdx.x + (threadIdx.x & 63);
    const int vb = threadIdx.x >> 6;
    const double* Vt = V + (int64_t)t * B * m;
    for (int e = threadIdx.x; e < 4 * m; e += 256) {
        const int bb = b0 + e / m;
        vs[e] = bb < B ? Vt[(int64_t)bb * m + e % m] : 0.0;
    }
    __syncthreads();
    const int b = b0 + vb;
    if (j >= n || b >= B) return;
    const double* row = Tt + ((int64_t)t * n + (n - 1 - j)) * m;     // T[.][j], reversed
    const double* v = vs + vb * m;
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc = fma(v[i], row[m - 1 - i], acc);
    I[((int64_t)t * B + b) * n + j] = acc;
}

Inner inner_of(const xbar_tile_class& c, double g_wl, double g_bl, double g_src, double g_sense)
{
    if (!c.transpose) return Inner{c.m, c.n, c.B, false, g_wl, g_bl, g_src, g_sense};
    return Inner{c.n, c.m, c.n, true, g_bl, g_wl, g_sense, g_src};
}

__global__ void tiles_clear_kernel(int* flags, unsigned long long* diag, int* bad, int T)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) bad[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < xbk::kNumFlags) flags[threadIdx.x] = 0;
    if (i == 0) diag[xbk::kDiagMinPivot] = xbk::kPivotKeyInf;
}

}  // namespace

struct xbar_tiles_s {
    std::vector<xbar_tile_class> cls;
    std::vector<PipeBuffers> pipe;
    std::vector<int> order;              // classes, most work first
    double g_wl = 0, g_bl = 0, g_src = 0, g_sense = 0;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    int device = 0;
    int64_t bytes = 0;
};

namespace {

void tiles_free(xbar_tiles t)
{
    for (PipeBuffers& b : t->pipe) {
        void* all[] = {b.H, b.c, b.fr, b.ip, b.q, b.Gc, b.S[0][0], b.S[0][1], b.S[1][0], b.S[1][1],
                       b.P[0][0], b.P[0][1], b.P[1][0], b.P[1][1], b.W[0], b.W[1], b.Z, b.flags, b.diag, b.sink,
                       b.bad, b.Gt, b.Tt};
        for (void* x : all)
            if (x) (void)hipFree(x);
        b = PipeBuffers{};
    }
    for (hipEvent_t e : t->join)
        if (e) (void)hipEventDestroy(e);
    if (t->fork) (void)hipEventDestroy(t->fork);
    for (hipStream_t s : t->side)
        if (s) (void)hipStreamDestroy(s);
    t->join.clear();
    t->side.clear();
    t->fork = nullptr;
}

// the class's work in flops (the method's count): factor m n^3, currents-only
// forward sweep 2 m n^2 per vector
double class_work(const xbar_tile_class& c)
{
    return (double)c.count * ((double)c.m * c.n * c.n * c.n + 2.0 * c.m * c.n * c.n * c.B);
}

hipError_t run_pipe(xbar_tiles t, int k, const Inner& in, const double* G, const double* V, double* I, hipStream_t s)
{
    const xbar_tile_class& c = t->cls[k];
    PipeBuffers& b = t->pipe[k];
    const int T = c.count, m = in.mi, n = in.ni, n_p = b.n_p;
    hipLaunchKernelGGL(tiles_clear_kernel, dim3((T + 255) / 256), dim3(256), 0, s, b.flags, b.diag, b.bad, T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    xbk::CondenseArgs ca{};
    ca.G = G;
    ca.m = m;
    ca.n = n;
    ca.n_p = n_p;
    ca.g_wl = in.g_wl;
    ca.g_bl = in.g_bl;
    ca.g_src = in.g_src;
    ca.g_sense = in.g_sense;
    ca.E = b.H;
    ca.c = b.c;
    ca.fr = b.fr;
    ca.ip = b.ip;
    ca.q = b.q;
    ca.Gc = b.Gc;
    ca.flags = b.flags;
    ca.tile_bad = b.bad;
    if ((e = xbk_launch_condense(ca, false, s, T)) != hipSuccess) return e;
    xbk::GJArgs ga{};
    ga.m = m;
    ga.n = n;
    ga.n_p = n_p;
    ga.nb = b.nb;
    ga.g2 = in.g_bl * in.g_bl;
    ga.H = b.H;
    for (int ch = 0; ch < 2; ++ch) {
        ga.job[ch].row = ga.job[ch].next = ga.job[ch].dep_a = ga.job[ch].dep_b = -1;
        for (int q = 0; q < 2; ++q) {
            ga.job[ch].S[q] = b.S[ch][q];
            ga.job[ch].P[q] = b.P[ch][q];
        }
        ga.job[ch].W = b.W[ch];      // warm starts of the pivot-tile inverses
    }
    ga.flags = b.flags;
    ga.diag = b.diag;
    ga.batch = T;
    ga.h_stride = (int64_t)m * n_p * n_p;
    ga.s_stride = (int64_t)n_p * n_p;
    ga.p_stride = (int64_t)xbk::kTile * xbk::kTile;
    ga.w_stride = (int64_t)2 * b.nb * xbk::kTile * xbk::kTile;
    ga.tile_bad = b.bad;
    if ((e = xbk_launch_factor(ga, false, s)) != hipSuccess) return e;
    xbk::SweepArgs sa{};
    sa.m = m;
    sa.n = n;
    sa.n_p = n_p;
    sa.B = in.Bi;
    sa.nslab = b.slabs;
    sa.g_bl = in.g_bl;
    sa.g_sense = in.g_sense;
    sa.H = b.H;
    sa.c = b.c;
    sa.V = V;
    sa.Z = b.Z;
    sa.Iout = I;
    sa.flags = b.flags;
    sa.sink = b.sink;
    sa.node_v = nullptr;
    sa.Gc = b.Gc;
    sa.fr = b.fr;
    sa.ip = b.ip;
    sa.g_src = in.g_src;
    sa.g_wl = in.g_wl;
    sa.unit = in.unit ? 1 : 0;
    sa.batch = T;
    sa.slabs_per = b.slabs;
    sa.tile_bad = b.bad;
    return xbk_launch_sweep(sa, s);
}

// One class on stream s: directly, or through its reciprocal problem and the product
// I = V T.
hipError_t run_class(xbar_tiles t, int k, const double* G, const double* V, double* I, hipStream_t s)
{
    const xbar_tile_class& c = t->cls[k];
    PipeBuffers& b = t->pipe[k];
    const Inner in = inner_of(c, t->g_wl, t->g_bl, t->g_src, t->g_sense);
    const double* Gi = G;
    double* Ii = I;
    hipError_t e;
    if (c.transpose) {
        const int64_t total = (int64_t)c.count * c.m * c.n;
        const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
        hipLaunchKernelGGL(rotate_transpose_kernel, dim3(grid), dim3(256), 0, s, G, b.Gt, c.count, c.m, c.n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        Gi = b.Gt;
        Ii = b.Tt;
    }
    if (c.method == XBAR_TILE_ONE_WG)
        e = xbk_launch_tile_currents(c.count, in.mi, in.ni, in.Bi, in.g_wl, in.g_bl, in.g_src, in.g_sense, Gi, V, Ii, s,
                                     c.block, c.split, in.unit);
    else
        e = run_pipe(t, k, in, Gi, V, Ii, s);
    if (e != hipSuccess || !c.transpose) return e;
    const dim3 grid((unsigned)((c.n + 63) / 64), (unsigned)((c.B + 3) / 4), (unsigned)c.count);
    hipLaunchKernelGGL(apply_reciprocal_kernel, grid, dim3(256), 4 * (size_t)c.m * sizeof(double), s, V, b.Tt, I, c.m,
                       c.n, c.B);
    return hipGetLastError();
}

}  // namespace

extern "C" {

xbar_status xbar_tiles_create(const xbar_tile_class* classes, int32_t nclasses, double r_wl, double r_bl,
                              double r_src, double r_sense, int32_t streams, void* hip_stream, xbar_tiles* out)
{
    if (out == nullptr || classes == nullptr || nclasses < 1 || streams < 1 || streams > 8) return XBAR_ERR_ARG;
    *out = nullptr;
    if (!finite_pos(r_wl) || !finite_pos(r_bl) || !finite_pos(r_src) || !finite_pos(r_sense)) return XBAR_ERR_ARG;
    for (int k = 0; k < nclasses; ++k) {
        const xbar_tile_class& c = classes[k];
        if (c.m < 1 || c.n < 1 || c.count < 1 || c.B < 1 || c.B > XBAR_TILE_MAX_B) return XBAR_ERR_ARG;
        if (c.transpose != 0 && c.transpose != 1) return XBAR_ERR_ARG;
        // the problem the kernels solve: the class, or its reciprocal with n unit inputs
        const int ni = c.transpose ? c.m : c.n, Bi = c.transpose ? c.n : c.B;
        if (Bi > XBAR_TILE_MAX_B) return XBAR_ERR_ARG;
        if (c.method == XBAR_TILE_ONE_WG) {
            if (ni > XBAR_TILE_MAX_N || c.split < 1 || c.split > 4) return XBAR_ERR_ARG;
            if (c.block != 0 && ((c.block != 16 && c.block != 32 && c.block != 64) || c.block < ni))
                return XBAR_ERR_ARG;
        } else if (c.method == XBAR_TILE_PIPELINE) {
            if (ni > XBAR_MAX_N || c.block != 0 || c.split != 1) return XBAR_ERR_ARG;
        } else {
            return XBAR_ERR_ARG;
        }
    }
    int ndev = 0, dev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return XBAR_ERR_DEVICE;
    }
    xbar_tiles t = new (std::nothrow) xbar_tiles_s;
    if (!t) return XBAR_ERR_ALLOC;
    t->cls.assign(classes, classes + nclasses);
    t->pipe.resize(nclasses);
    t->g_wl = 1.0 / r_wl;
    t->g_bl = 1.0 / r_bl;
    t->g_src = 1.0 / r_src;
    t->g_sense = 1.0 / r_sense;
    t->stream = reinterpret_cast<hipStream_t>(hip_stream);
    t->device = dev;
    xbar_status st = XBAR_OK;
    auto A = [&](void** p, int64_t bytes) {
        if (st != XBAR_OK) return;
        if (hipMalloc(p, (size_t)std::max<int64_t>(bytes, 256)) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            st = XBAR_ERR_ALLOC;
            return;
        }
        t->bytes += bytes;
    };
    for (int k = 0; k < nclasses && st == XBAR_OK; ++k) {
        const xbar_tile_class& c = classes[k];
        PipeBuffers& b = t->pipe[k];
        if (c.transpose) {
            A((void**)&b.Gt, (int64_t)c.count * c.m * c.n * 8);
            A((void**)&b.Tt, (int64_t)c.count * c.m * c.n * 8);
        }
        if (c.method != XBAR_TILE_PIPELINE) continue;
        const Inner in = inner_of(c, 1, 1, 1, 1);
        const int64_t T = c.count, m = in.mi, n = in.ni;
        b.n_p = 64 * ((in.ni + 63) / 64);
        b.nb = b.n_p / 64;
        b.slabs = (in.Bi + 15) / 16;
        const int64_t n_p = b.n_p;
        A(&b.H, T * m * n_p * n_p * 8);
        A((void**)&b.c, T * m * n_p * 8);
        A((void**)&b.fr, T * m * n * 8);
        A((void**)&b.ip, T * m * n * 8);
        A((void**)&b.q, T * m * n * 8);
        A((void**)&b.Gc, T * m * n * 8);
        for (int ch = 0; ch < 2; ++ch) {
            for (int q = 0; q < 2; ++q) {
                A(&b.S[ch][q], T * n_p * n_p * 8);
                A(&b.P[ch][q], T * xbk::kTile * xbk::kTile * 8);
            }
            // Newton-Schulz pivot tiles pay where a launch waits on its pivot inversions:
            // up to kNsPivotJobs jobs (a launch has one inversion per job).  Larger
            // batches fill the chip with updates, and the round's four products cost
            // more than the elimination (1024 maps of 128 x 128: 8.6k against 9.8k
            // maps/s); without slots every pivot tile is eliminated.
            if (2 * T <= kNsPivotJobs) A(&b.W[ch], T * 2 * b.nb * xbk::kTile * xbk::kTile * 8);
        }
        A(&b.Z, T * b.slabs * m * 16 * n_p * 8);
        A((void**)&b.flags, xbk::kNumFlags * sizeof(int));
        A((void**)&b.diag, xbk::kNumDiag * sizeof(unsigned long long));
        A((void**)&b.sink, 128 * sizeof(double));
        A((void**)&b.bad, T * sizeof(int));
    }
    if (st == XBAR_OK) {
        t->side.assign(streams, nullptr);
        t->join.assign(streams, nullptr);
        if (hipEventCreateWithFlags(&t->fork, hipEventDisableTiming) != hipSuccess) st = XBAR_ERR_DEVICE;
        for (int j = 0; j < streams && st == XBAR_OK; ++j)
            if (hipStreamCreateWithFlags(&t->side[j], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&t->join[j], hipEventDisableTiming) != hipSuccess)
                st = XBAR_ERR_DEVICE;
    }
    if (st != XBAR_OK) {
        (void)hipGetLastError();
        tiles_free(t);
        delete t;
        return st;
    }
    t->order.resize(nclasses);
    for (int k = 0; k < nclasses; ++k) t->order[k] = k;
    std::stable_sort(t->order.begin(), t->order.end(),
                     [&](int a, int b) { return class_work(t->cls[a]) > class_work(t->cls[b]); });
    *out = t;
    return XBAR_OK;
}

xbar_status xbar_tiles_run(xbar_tiles t, const double* const* G, const double* const* V, double* const* I)
{
    if (t == nullptr || G == nullptr || V == nullptr || I == nullptr) return XBAR_ERR_ARG;
    const int nc = (int)t->cls.size();
    for (int k = 0; k < nc; ++k)
        if (G[k] == nullptr || V[k] == nullptr || I[k] == nullptr) return XBAR_ERR_ARG;
    if (hipSetDevice(t->device) != hipSuccess) return XBAR_ERR_DEVICE;
    const int ns = (int)t->side.size();
    if (hipEventRecord(t->fork, t->stream) != hipSuccess) return XBAR_ERR_DEVICE;
    for (int j = 0; j < ns; ++j)
        if (hipStreamWaitEvent(t->side[j], t->fork, 0) != hipSuccess) return XBAR_ERR_DEVICE;
    // classes round-robin over the streams, most work first
    for (int j = 0; j < nc; ++j) {
        const int k = t->order[j];
        hipStream_t s = t->side[j % ns];
        const hipError_t e = run_class(t, k, G[k], V[k], I[k], s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return XBAR_ERR_DEVICE;
        }
    }
    for (int j = 0; j < ns; ++j)
        if (hipEventRecord(t->join[j], t->side[j]) != hipSuccess ||
            hipStreamWaitEvent(t->stream, t->join[j], 0) != hipSuccess)
            return XBAR_ERR_DEVICE;
    return XBAR_OK;
}

int64_t xbar_tiles_workspace_bytes(xbar_tiles t)
{
    return t == nullptr ? -1 : t->bytes;
}

xbar_status xbar_tiles_destroy(xbar_tiles t)
{
    if (t == nullptr) return XBAR_OK;
    (void)hipSetDevice(t->device);
    (void)hipStreamSynchronize(t->stream);
    for (hipStream_t s : t->side)
        if (s) (void)hipStreamSynchronize(s);
    tiles_free(t);
    delete t;
    return XBAR_OK;
}

}  // extern "C"

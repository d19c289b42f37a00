// C ABI of the crossbar solver: plan lifetime, host-side validation,
// workspace sizing and the call-order state machine (include/xbar.h).
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "tiles.h"
#include "transfer.h"
#include "xbar.h"

namespace {

enum State : int32_t { kCreated = 0, kAssembled = 1, kFactored = 2, kSolved = 3 };

struct Buffers {
    void* H = nullptr;        // [m][n_p][n_p] E_i, then H_i (factor precision)
    double* c = nullptr;      // [m][n_p]
    double* fr = nullptr;     // [m][n]
    double* ip = nullptr;     // [m][n]
    double* q = nullptr;      // [m][n]
    double* Gc = nullptr;     // [m][n]
    void* S[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [chain][parity]
    void* P[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    void* Z = nullptr;        // [nslab][m][16][n_p]
    double* Iout = nullptr;   // [max_batch][n]
    int* flags = nullptr;     // [kNumFlags]
    unsigned long long* diag = nullptr;   // [kNumDiag]: smallest pivot key, largest backward error bits
    double* sink = nullptr;   // [128]: target of the sweep's L2-pull keep-alive store
    // Newton-Schulz factor: per chain S, X[2], Q ([n_p][n_p]) and dprev ([2][n_p])
    void* ns_S[2] = {nullptr, nullptr};
    void* ns_X[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    void* ns_Q[2] = {nullptr, nullptr};
    double* ns_dprev[2] = {nullptr, nullptr};
    double* ns_part = nullptr;               // [2][(n_p/32)^2]
    xbk::NSState* ns_state = nullptr;        // [2 parities][3 schedules] schedule state
    // refinement (IR modes): float64 solutions, float residual panels, per-slab state
    double* U[2] = {nullptr, nullptr};       // [nslab][m][16][n_p]
    void* R = nullptr;                       // [nslab][m][16][n_p] float
    double* dnorm = nullptr;                 // [nslab][16]
    int* slab_done = nullptr;                // [nslab]
    int* slab_final = nullptr;               // [nslab]
    double* Vunit = nullptr;                 // [tr_rows][m]: unit inputs of xbar_transfer (plans
                                             // without the block form only)
    // Krylov refinement (XBAR_BF16_GMRES_IR): Arnoldi basis v_0..v_k and preconditioned
    // directions z_0..z_{k-1} (panels), a zero panel, reduction partials, the Hessenberg
    // matrices [k+1][k][Bp], beta [Bp], y [k][Bp] and Gram-Schmidt coefficients [k+1][Bp]
    double* gm_V = nullptr;
    double* gm_Z = nullptr;
    double* gm_zero = nullptr;
    double* gm_part = nullptr;
    double* gm_H = nullptr;
    double* gm_beta = nullptr;
    double* gm_y = nullptr;
    double* gm_coef = nullptr;
    // reciprocal ordering: the reciprocal crossbar's conductances [m][n] and its node
    // voltages [max_batch][2mn] (always recovered: the given crossbar's currents are the
    // reciprocal's first word-line nodes)
    double* Grev = nullptr;
    double* nv_rev = nullptr;
};

__global__ void clear_slabs_kernel(int* done, double* dnorm, int nslab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nslab) done[i] = 0;
    if (i < 16 * nslab) dnorm[i] = 0.0;
}

__global__ void clear_flags_kernel(int* f)
{
    if (threadIdx.x < xbk::kNumFlags) f[threadIdx.x] = 0;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

// HIP-event timer of one kernel phase: event pairs recorded around launches and
// resolved lazily (no synchronisation on the launch path).
struct PhaseTimer {
    std::vector<hipEvent_t> ev;     // pairs (start, stop), reused
    size_t used = 0;                 // events in use
    double ms = 0.0;
    int64_t launches = 0;
    bool begin(hipStream_t s) {
        if (used + 2 > ev.size()) {
            if (!flush()) return false;
            if (ev.size() < 2 * 256) {
                hipEvent_t a, b;
                if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return false;
                ev.push_back(a);
                ev.push_back(b);
            }
        }
        return hipEventRecord(ev[used], s) == hipSuccess;
    }
    bool end(hipStream_t s) {
        if (hipEventRecord(ev[used + 1], s) != hipSuccess) return false;
        used += 2;
        return true;
    }
    bool flush() {
        for (size_t k = 0; k + 1 < used; k += 2) {
            float t = 0.f;
            if (hipEventSynchronize(ev[k + 1]) != hipSuccess) return false;
            if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) != hipSuccess) return false;
            ms += t;
            ++launches;
        }
        used = 0;
        return true;
    }
    void destroy() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        used = 0;
    }
};

struct xbar_plan_s {
    // g: the crossbar the solver works on; og: the crossbar as given.  They differ in
    // reciprocal ordering (og.n > og.m): then g is og rotated by 180 degrees and
    // transposed (g.m = og.n, g.n = og.m, word and bit lines exchanged, r_src and
    // r_sense exchanged), so that the row blocks have the smaller size og.m.
    xbar_geometry g{};
    xbar_geometry og{};
    bool rev = false;
    xbar_precision prec = XBAR_FP64;
    int32_t max_batch = 0;
    double ir_tol = 0;
    int32_t ir_max_iter = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int n_p = 0, nb = 0, nslab_max = 0;
    int tr_rows = 0;                    // unit inputs per xbar_transfer solve: min(max_batch, m)
    int64_t bytes = 0;
    int32_t state = kCreated;
    int32_t last_B = 0;
    Buffers d;
    bool timing = false;
    int32_t factor_method = XBAR_FACTOR_AUTO;
    int64_t gj_fallbacks = 0;
    int ns_slots_hint[3] = {0, 0, 0};   // slots each Newton-Schulz schedule last needed (checked mode)
    int ns_launched[3] = {0, 0, 0};     // slots the last Newton-Schulz factorization launched
    int ns_used_host = 0;               // slots used, when the factorization read its states back
    bool ns_hint_valid = false;         // ns_slots_hint holds what the last factorization needed
    bool ns_async = false;              // the last factorization ran the asynchronous schedule
    double pivot_shift = 0.0;           // test hook: subtracted from diag(E_i) at assembly
    bool diagnostics = false;           // measure the backward error of solved batches
    bool backerr_valid = false;         // the last solve measured it
    hipStream_t side = nullptr;         // second stream: the bottom chain of the factor
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    PhaseTimer t_condense, t_factor, t_sweep, t_recover, t_ir_sweep, t_residual;
    bool fp32() const { return prec != XBAR_FP64; }
    size_t elem() const { return fp32() ? sizeof(float) : sizeof(double); }
};

namespace {

xbar_status dev_alloc(xbar_plan p, void** ptr, int64_t bytes)
{
    if (bytes <= 0) bytes = 256;
    if (hipMalloc(ptr, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return XBAR_ERR_ALLOC;
    }
    p->bytes += bytes;
    return XBAR_OK;
}

void free_all(xbar_plan p)
{
    Buffers& d = p->d;
    void* all[] = {d.H, d.c, d.fr, d.ip, d.q, d.Gc, d.S[0][0], d.S[0][1], d.S[1][0], d.S[1][1],
                   d.P[0][0], d.P[0][1], d.P[1][0], d.P[1][1], d.Z, d.Iout, d.flags, d.diag, d.sink,
                   d.ns_S[0], d.ns_S[1], d.ns_X[0][0], d.ns_X[0][1], d.ns_X[1][0], d.ns_X[1][1],
                   d.ns_Q[0], d.ns_Q[1],
                   d.ns_dprev[0], d.ns_dprev[1], d.ns_part, d.ns_state,
                   d.U[0], d.U[1], d.R, d.dnorm, d.slab_done, d.slab_final, d.Vunit,
                   d.gm_V, d.gm_Z, d.gm_zero, d.gm_part, d.gm_H, d.gm_beta, d.gm_y, d.gm_coef,
                   d.Grev, d.nv_rev};
    for (void* x : all)
        if (x) (void)hipFree(x);
    d = Buffers{};
}

bool set_device(xbar_plan p) { return hipSetDevice(p->device) == hipSuccess; }

// The block form of xbar_transfer keeps m FRG blocks of n_p x n_p in the sweep workspace
// (float64 plans whose max_batch, rounded up to 16, is at least n_p); other plans solve
// unit inputs and hold a staging buffer for them.
// Cost model of the choice between the two orderings of an m x n crossbar with n > m.
// A simulation (assembly, factor, solve) walks the chain of row blocks in sequence,
// at about t(n_p) microseconds per row for the padded block size n_p; measured on
// gfx950 (float64, one to 256 input vectors) the cost is nearly flat up to n_p = 128
// and grows beyond: t = 14, 15, 22, 30, 42, 55, 67, 80 for n_p = 64 .. 512.  Rows:
// m t(pad(n)); reciprocal: n t(pad(m)).  With it, among the wide shapes up to 256 x 512
// the reciprocal wins at 128 x 512 and 256 x 512 and loses at every smaller or narrower
// one, as the measurements did.
double row_us(int n)
{
    const int n_p = 64 * ((n + 63) / 64);
    static const double t[9] = {0.0, 14.0, 15.0, 22.0, 30.0, 42.0, 55.0, 67.0, 80.0};   // n_p = 64 k
    return t[n_p / 64];
}

bool reciprocal_is_faster(int m, int n)
{
    if (n > XBAR_MAX_N) return true;
    return (double)n * row_us(m) < (double)m * row_us(n);
}

bool transfer_blocks_fit(xbar_plan p)
{
    return !p->rev && p->prec == XBAR_FP64 && (int64_t)p->nslab_max * 16 >= p->n_p;
}

// Reciprocal crossbar of the given m x n one (n > m): Gr [n][m], Gr[i][j] = G[m-1-j][n-1-i].
__global__ void rev_conductances_kernel(const double* __restrict__ G, int m, int n, double* __restrict__ Gr)
{
    const int64_t total = (int64_t)m * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / m, j = e - i * m;
        Gr[e] = G[(m - 1 - j) * (int64_t)n + (n - 1 - i)];
    }
}

// Outputs of the given crossbar (m x n, n > m) from the reciprocal's node voltages
// nr [B][2 n m]: column j's current flows through the sense resistor at BL(m-1, j),
// which is the reciprocal's source resistor at its WL(n-1-j, 0); node WL(i, j) of the
// given crossbar is the reciprocal's BL(n-1-j, m-1-i) and BL(i, j) its WL(n-1-j, m-1-i).
// I [B][n]; node_v [B][2mn] (paper order) when not null.
__global__ void rev_outputs_kernel(const double* __restrict__ nr, int B, int m, int n, double g_sense,
                                   double* __restrict__ I, double* __restrict__ node_v)
{
    const int64_t per = (int64_t)m * n;
    const int64_t total = (int64_t)B * per;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / per, r = e - b * per;
        const int i = (int)(r / n), j = (int)(r - (int64_t)i * n);
        const int64_t rr = (int64_t)(n - 1 - j) * m + (m - 1 - i);          // reciprocal's (row, column)
        const double* x = nr + b * 2 * per;
        if (node_v) {
            node_v[b * 2 * per + 2 * r] = x[2 * rr + 1];
            node_v[b * 2 * per + 2 * r + 1] = x[2 * rr];
        }
        if (i == m - 1) I[b * n + j] = g_sense * x[2 * rr];       // reciprocal WL(n-1-j, 0)
    }
}

unsigned grid_for(int64_t count)
{
    const int64_t blocks = (count + 255) / 256;
    return (unsigned)(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192);
}

void destroy_side(xbar_plan p)
{
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->side) (void)hipStreamDestroy(p->side);
    p->ev_join = p->ev_fork = nullptr;
    p->side = nullptr;
}

xbk::CondenseArgs condense_args(xbar_plan p, const double* G);

// Condensation of the rows (A1 + A2) into the plan's E blocks, then the test
// hook's diagonal shift when one is set.
hipError_t condense(xbar_plan p, const double* G)
{
    hipError_t e = xbk_launch_condense(condense_args(p, G), p->fp32(), p->stream);
    if (e == hipSuccess && p->pivot_shift != 0.0)
        e = xbk_launch_shift_diag(p->d.H, p->fp32(), p->g.m, p->g.n, p->n_p, p->pivot_shift, p->stream);
    return e;
}

}  // namespace

extern "C" {

const char* xbar_status_string(xbar_status s)
{
    switch (s) {
        case XBAR_OK: return "XBAR_OK";
        case XBAR_ERR_ARG: return "XBAR_ERR_ARG";
        case XBAR_ERR_ALLOC: return "XBAR_ERR_ALLOC";
        case XBAR_ERR_STATE: return "XBAR_ERR_STATE";
        case XBAR_ERR_NOT_SPD: return "XBAR_ERR_NOT_SPD";
        case XBAR_ERR_NO_CONVERGENCE: return "XBAR_ERR_NO_CONVERGENCE";
        case XBAR_ERR_DEVICE: return "XBAR_ERR_DEVICE";
        case XBAR_ERR_INPUT: return "XBAR_ERR_INPUT";
    }
    return "XBAR_UNKNOWN_STATUS";
}

xbar_status xbar_create(const xbar_geometry* geom, xbar_precision prec, int32_t max_batch,
                        double ir_tol, int32_t ir_max_iter, void* hip_stream, xbar_plan* out)
{
    return xbar_create_ordered(geom, prec, max_batch, ir_tol, ir_max_iter, hip_stream, XBAR_ORDER_AUTO, out);
}

xbar_status xbar_create_ordered(const xbar_geometry* geom, xbar_precision prec, int32_t max_batch,
                                double ir_tol, int32_t ir_max_iter, void* hip_stream, int32_t ordering,
                                xbar_plan* out)
{
    if (out == nullptr || geom == nullptr) return XBAR_ERR_ARG;
    *out = nullptr;
    const xbar_geometry og = *geom;
    if (og.m < 1 || og.n < 1 || std::min(og.m, og.n) > XBAR_MAX_N) return XBAR_ERR_ARG;
    if (!finite_pos(og.r_wl) || !finite_pos(og.r_bl) || !finite_pos(og.r_src) || !finite_pos(og.r_sense))
        return XBAR_ERR_ARG;
    if (ordering != XBAR_ORDER_AUTO && ordering != XBAR_ORDER_ROWS && ordering != XBAR_ORDER_SMALLER)
        return XBAR_ERR_ARG;
    if (ordering == XBAR_ORDER_ROWS && og.n > XBAR_MAX_N) return XBAR_ERR_ARG;
    // reciprocal ordering: the crossbar turned by 180 degrees and transposed, so that the
    // row blocks take the smaller side m
    const bool rev = og.n > og.m && (ordering == XBAR_ORDER_SMALLER ||
                                     (ordering == XBAR_ORDER_AUTO && reciprocal_is_faster(og.m, og.n)));
    xbar_geometry g = og;
    if (rev) {
        g.m = og.n;
        g.n = og.m;
        g.r_wl = og.r_bl;
        g.r_bl = og.r_wl;
        g.r_src = og.r_sense;
        g.r_sense = og.r_src;
    }
    if (prec != XBAR_FP64 && prec != XBAR_FP32_IR && prec != XBAR_BF16_IR && prec != XBAR_BF16_GMRES_IR)
        return XBAR_ERR_ARG;
    if (max_batch < 1) return XBAR_ERR_ARG;
    if (!(std::isfinite(ir_tol) && ir_tol >= 0.0 && ir_tol < 1.0)) return XBAR_ERR_ARG;
    if (ir_max_iter < 0 || ir_max_iter > 100) return XBAR_ERR_ARG;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return XBAR_ERR_DEVICE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return XBAR_ERR_DEVICE;

    xbar_plan p = new (std::nothrow) xbar_plan_s;
    if (!p) return XBAR_ERR_ALLOC;
    p->g = g;
    p->og = og;
    p->rev = rev;
    p->prec = prec;
    p->max_batch = max_batch;
    p->ir_tol = (ir_tol == 0.0) ? 1e-12 : ir_tol;
    p->ir_max_iter = (ir_max_iter == 0) ? 10 : ir_max_iter;
    p->stream = reinterpret_cast<hipStream_t>(hip_stream);
    p->device = dev;
    p->n_p = 64 * ((g.n + 63) / 64);
    p->nb = p->n_p / 64;
    p->nslab_max = (max_batch + 15) / 16;
    p->tr_rows = max_batch < og.m ? max_batch : og.m;

    const int64_t m = g.m, n = g.n, n_p = p->n_p, es = (int64_t)p->elem();
    Buffers& d = p->d;
    xbar_status st = XBAR_OK;
    auto A = [&](void** ptr, int64_t bytes) {
        if (st == XBAR_OK) st = dev_alloc(p, ptr, bytes);
    };
    A(&d.H, m * n_p * n_p * es);
    A((void**)&d.c, m * n_p * 8);
    A((void**)&d.fr, m * n * 8);
    A((void**)&d.ip, m * n * 8);
    A((void**)&d.q, m * n * 8);
    A((void**)&d.Gc, m * n * 8);
    for (int c = 0; c < 2; ++c)
        for (int k = 0; k < 2; ++k) {
            A(&d.S[c][k], n_p * n_p * es);
            A(&d.P[c][k], 64 * 64 * es);
        }
    A(&d.Z, (int64_t)p->nslab_max * m * 16 * n_p * es);
    A((void**)&d.Iout, (int64_t)max_batch * og.n * 8);
    A((void**)&d.flags, xbk::kNumFlags * sizeof(int));
    A((void**)&d.diag, xbk::kNumDiag * sizeof(unsigned long long));
    A((void**)&d.sink, 128 * sizeof(double));
    for (int c = 0; c < 2; ++c) {
        A(&d.ns_S[c], n_p * n_p * es);
        A(&d.ns_X[c][0], n_p * n_p * es);
        A(&d.ns_X[c][1], n_p * n_p * es);
        A(&d.ns_Q[c], n_p * n_p * es);
        A((void**)&d.ns_dprev[c], 2 * n_p * 8);
    }
    A((void**)&d.ns_part, 2 * (n_p / 32) * (n_p / 32) * 8);
    A((void**)&d.ns_state, 6 * sizeof(xbk::NSState));
    if (!transfer_blocks_fit(p)) A((void**)&d.Vunit, (int64_t)p->tr_rows * og.m * 8);
    if (rev) {
        A((void**)&d.Grev, m * n * 8);
        A((void**)&d.nv_rev, (int64_t)max_batch * 2 * m * n * 8);
    }
    if (prec != XBAR_FP64) {
        const int64_t panel = (int64_t)p->nslab_max * m * 16 * n_p;
        A((void**)&d.U[0], panel * 8);
        A((void**)&d.U[1], panel * 8);
        A(&d.R, panel * 4);
        A((void**)&d.dnorm, (int64_t)p->nslab_max * 16 * 8);
        A((void**)&d.slab_done, (int64_t)p->nslab_max * 4);
        A((void**)&d.slab_final, (int64_t)p->nslab_max * 4);
        if (prec == XBAR_BF16_GMRES_IR) {
            constexpr int K = xbk::kGmRestart;
            const int64_t Bp = 16 * (int64_t)p->nslab_max;
            A((void**)&d.gm_V, (K + 1) * panel * 8);
            A((void**)&d.gm_Z, K * panel * 8);
            A((void**)&d.gm_zero, panel * 8);
            A((void**)&d.gm_part, (int64_t)m * (K + 1) * Bp * 8);     // at most m chunks
            A((void**)&d.gm_H, (int64_t)(K + 1) * K * Bp * 8);
            A((void**)&d.gm_beta, Bp * 8);
            A((void**)&d.gm_y, K * Bp * 8);
            A((void**)&d.gm_coef, (K + 1) * Bp * 8);
            if (st == XBAR_OK && xbk_gm_fill(d.gm_zero, panel, 0.0, p->stream) != hipSuccess) st = XBAR_ERR_DEVICE;
        }
    }
    if (st != XBAR_OK) {
        free_all(p);
        delete p;
        return st;
    }
    hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(64), 0, p->stream, d.flags);
    if (hipGetLastError() != hipSuccess || xbk_launch_reset_diag(d.diag, 3, p->stream) != hipSuccess ||
        hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        destroy_side(p);
        free_all(p);
        delete p;
        return XBAR_ERR_DEVICE;
    }
    *out = p;
    return XBAR_OK;
}

xbar_status xbar_assemble(xbar_plan p, const double* G)
{
    if (p == nullptr || G == nullptr) return XBAR_ERR_ARG;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(64), 0, p->stream, p->d.flags);
    if (xbk_launch_reset_diag(p->d.diag, 3, p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
    p->backerr_valid = false;
    if (p->timing && !p->t_condense.begin(p->stream)) return XBAR_ERR_DEVICE;
    if (p->rev) {
        hipLaunchKernelGGL(rev_conductances_kernel, dim3(grid_for((int64_t)p->og.m * p->og.n)), dim3(256), 0,
                           p->stream, G, p->og.m, p->og.n, p->d.Grev);
        if (hipGetLastError() != hipSuccess) return XBAR_ERR_DEVICE;
        G = p->d.Grev;
    }
    if (condense(p, G) != hipSuccess) return XBAR_ERR_DEVICE;
    if (p->timing && !p->t_condense.end(p->stream)) return XBAR_ERR_DEVICE;
    p->state = kAssembled;
    return XBAR_OK;
}

}  // extern "C"

namespace {

xbk::CondenseArgs condense_args(xbar_plan p, const double* G)
{
    xbk::CondenseArgs a{};
    a.G = G;
    a.m = p->g.m;
    a.n = p->g.n;
    a.n_p = p->n_p;
    a.g_wl = 1.0 / p->g.r_wl;
    a.g_bl = 1.0 / p->g.r_bl;
    a.g_src = 1.0 / p->g.r_src;
    a.g_sense = 1.0 / p->g.r_sense;
    a.E = p->d.H;
    a.c = p->d.c;
    a.fr = p->d.fr;
    a.ip = p->d.ip;
    a.q = p->d.q;
    a.Gc = p->d.Gc;
    a.flags = p->d.flags;
    return a;
}

hipError_t launch_gj(xbar_plan p)
{
    xbk::GJArgs a{};
    a.m = p->g.m;
    a.n = p->g.n;
    a.n_p = p->n_p;
    a.nb = p->nb;
    const double gb = 1.0 / p->g.r_bl;
    a.g2 = gb * gb;
    a.H = p->d.H;
    for (int c = 0; c < 2; ++c) {
        a.job[c].row = a.job[c].next = a.job[c].dep_a = a.job[c].dep_b = -1;
        for (int k = 0; k < 2; ++k) {
            a.job[c].S[k] = p->d.S[c][k];
            a.job[c].P[k] = p->d.P[c][k];
        }
    }
    a.flags = p->d.flags;
    a.diag = p->d.diag;
    return xbk_launch_factor(a, p->fp32(), p->stream);
}

xbk::NSArgs ns_args(xbar_plan p)
{
    xbk::NSArgs a{};
    a.m = p->g.m;
    a.n = p->g.n;
    a.n_p = p->n_p;
    const double gb = 1.0 / p->g.r_bl;
    a.g2 = gb * gb;
    a.H = p->d.H;
    for (int c = 0; c < 2; ++c) {
        a.ch[c].S = p->d.ns_S[c];
        a.ch[c].X[0] = p->d.ns_X[c][0];
        a.ch[c].X[1] = p->d.ns_X[c][1];
        a.ch[c].Q = p->d.ns_Q[c];
        a.ch[c].dprev = p->d.ns_dprev[c];
    }
    a.state = p->d.ns_state;
    a.part = p->d.ns_part;
    a.flags = p->d.flags;
    a.diag = p->d.diag;
    a.max_iter = xbk::kNsMaxIter;
    return a;
}

// Launch budget of a Newton-Schulz schedule that is not read back: the launches
// it needed the last time they were read back (ns_slots_hint), plus a margin of
// extra rounds (three launches each in float64, one two-launch step in float32)
// for a conductance map whose rows need more.  The margin grows with the rounds
// beyond one per row that the schedule needed then (k): rows that need one or two
// rounds make the count vary from map to map by about sqrt(k) rounds.  Launches
// past a schedule's end only carry its final state over.
int ns_budget(xbar_plan p, int c)
{
    const int m = p->g.m, kt = m / 2;
    const int rows = c == 0 ? kt : c == 1 ? std::max(0, m - 1 - kt) : 1;
    if (rows == 0) return 0;
    const int per_round = p->fp32() ? 2 : 3;
    const double k = std::max(0.0, (p->ns_slots_hint[c] - 1) / (double)per_round - rows);
    const int margin = 4 + (int)std::ceil(0.5 * k + 4.0 * std::sqrt(k));
    return p->ns_slots_hint[c] + per_round * margin;
}

// Newton-Schulz factor on its device-driven schedule.  The two chains run on the
// plan stream and the side stream (so that one chain's launches fill the matrix
// cores while the other's start up or write out); schedule 2 (the twist) runs on
// the plan stream once both have finished.
//  - asynchronous (checked == false): each schedule gets its launch budget and
//    nothing is read back, so the call can be captured into a graph; a finishing
//    kernel raises kErrConv when a row missed its tolerance or a schedule ran out
//    of launches.
//  - checked: launch the slots the last factorization needed (or an estimate),
//    read the states back, and launch more until every schedule has finished;
//    *failed reports a missed tolerance or the cap.
hipError_t run_ns(xbar_plan p, bool checked, bool* failed)
{
    const xbk::NSArgs a = ns_args(p);
    *failed = false;
    hipError_t e = xbk_launch_ns_init(a, p->stream);
    if (e != hipSuccess) return e;
    const int m = p->g.m, kt = m / 2;
    const int rows[3] = {kt, std::max(0, m - 1 - kt), 1};
    hipStream_t on[3] = {p->stream, p->side, p->stream};
    int launched[3] = {0, 0, 0}, batch[3];
    int cap[3];
    for (int c = 0; c < 3; ++c) {
        const int steps = (c == 0 || c == 1) ? xbk::kNsMaxIter : xbk::kNsMaxIter + 4;
        cap[c] = rows[c] * (1 + 2 * (steps + 4)) + 4;
        if (!checked)
            batch[c] = ns_budget(p, c);
        else
            batch[c] = rows[c] == 0                ? 0
                       : p->ns_slots_hint[c] > 0 ? p->ns_slots_hint[c]
                       : c == 2                  ? 2 * steps + 2
                                                 : rows[c] * 5 + 8;
    }
    xbk::NSState st[6];
    int fail = 0;
    // read every state back (through the plan stream, after the side stream's work)
    auto sync_states = [&]() -> hipError_t {
        hipError_t r;
        if ((r = hipEventRecord(p->ev_join, p->side)) != hipSuccess ||
            (r = hipStreamWaitEvent(p->stream, p->ev_join, 0)) != hipSuccess ||
            (r = hipMemcpyAsync(st, p->d.ns_state, sizeof(st), hipMemcpyDeviceToHost, p->stream)) != hipSuccess ||
            (r = hipMemcpyAsync(&fail, p->d.flags + xbk::kNsFail, sizeof(int), hipMemcpyDeviceToHost,
                                p->stream)) != hipSuccess)
            return r;
        return hipStreamSynchronize(p->stream);
    };
    auto state_of = [&](int c) -> const xbk::NSState& { return st[3 * (launched[c] & 1) + c]; };
    // the side stream starts after the plan stream's work so far (E blocks, initial states)
    if ((e = hipEventRecord(p->ev_fork, p->stream)) != hipSuccess ||
        (e = hipStreamWaitEvent(p->side, p->ev_fork, 0)) != hipSuccess)
        return e;
    for (int phase = 0; phase < 2; ++phase) {
        const int c0 = phase == 0 ? 0 : 2, c1 = phase == 0 ? 1 : 2;
        for (;;) {
            // interleave the two chains' launches so that both streams stay fed
            const int most = std::max(batch[c0], batch[c1]);
            for (int k = 0; k < most; ++k)
                for (int c = c0; c <= c1; ++c)
                    if (k < batch[c] && (e = xbk_launch_ns_slots(a, p->fp32(), c, launched[c] + k, 1, on[c])) !=
                                            hipSuccess)
                        return e;
            for (int c = c0; c <= c1; ++c) launched[c] += batch[c];
            if (!checked) {
                if (phase == 0 &&
                    ((e = hipEventRecord(p->ev_join, p->side)) != hipSuccess ||
                     (e = hipStreamWaitEvent(p->stream, p->ev_join, 0)) != hipSuccess))
                    return e;
                break;
            }
            if ((e = sync_states()) != hipSuccess) return e;
            bool done = true, over = false;
            for (int c = c0; c <= c1; ++c) {
                const xbk::NSState& s = state_of(c);
                batch[c] = 0;
                if (s.phase == xbk::kNsFinished) continue;
                done = false;
                if (launched[c] >= cap[c]) {
                    over = true;
                    continue;
                }
                const int left = c == 0 ? kt - s.row : c == 1 ? s.row - kt : 1;
                batch[c] = std::min(std::max(8, 5 * left + 4), cap[c] - launched[c]);
            }
            if (over) {
                *failed = true;
                for (int c = 0; c < 3; ++c) p->ns_launched[c] = launched[c];
                return hipSuccess;
            }
            if (done) break;
        }
    }
    for (int c = 0; c < 3; ++c) p->ns_launched[c] = launched[c];
    if (!checked) return xbk_launch_ns_finish(a, launched[0], launched[1], launched[2], p->stream);
    p->ns_used_host = 0;
    for (int c = 0; c < 3; ++c) {
        p->ns_slots_hint[c] = state_of(c).slots;
        p->ns_used_host += state_of(c).slots;
    }
    *failed = fail != 0;
    p->ns_hint_valid = true;
    return hipSuccess;
}

__global__ void clear_flag_kernel(int* f, int which) { f[which] = 0; }

// The bfloat16 trial: round every stored inverse block to the nearest bfloat16
// value (8-bit significand, ties to even), kept in float32 storage.  NaN stays NaN.
__global__ void round_bf16_kernel(float* x, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[e];
        if (v != v) continue;
        uint32_t u = __float_as_uint(v);
        u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
        x[e] = __uint_as_float(u);
    }
}
__global__ void set_flag_kernel(int* f, int which) { f[which] = 1; }

// rows unit input vectors: V[b][i] = 1 if i == i0 + b else 0, b < rows
__global__ void unit_inputs_kernel(double* V, int rows, int m, int i0)
{
    const int64_t total = (int64_t)rows * m;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / m, i = e - b * m;
        V[e] = (i == i0 + b) ? 1.0 : 0.0;
    }
}

bool overlaps(const void* a, int64_t a_bytes, const void* b, int64_t b_bytes)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + (uintptr_t)b_bytes && y < x + (uintptr_t)a_bytes;
}

// T from the m unit input vectors, solved with the plan's factorization (any plan).
xbar_status transfer_by_unit_solves(xbar_plan p, double* T)
{
    const int m = p->og.m, n = p->og.n;                  // the crossbar as given
    const bool timing = p->timing;
    p->timing = false;                     // the unit solves are not counted as sweeps
    xbar_status st = XBAR_OK;
    for (int i0 = 0; i0 < m && st == XBAR_OK; i0 += p->tr_rows) {
        const int rows = p->tr_rows < m - i0 ? p->tr_rows : m - i0;
        const int64_t total = (int64_t)rows * m;
        const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
        hipLaunchKernelGGL(unit_inputs_kernel, dim3(grid), dim3(256), 0, p->stream, p->d.Vunit, rows, m, i0);
        if (hipGetLastError() != hipSuccess) {
            st = XBAR_ERR_DEVICE;
            break;
        }
        st = xbar_solve_batch(p, p->d.Vunit, rows, nullptr);
        if (st == XBAR_OK &&
            hipMemcpyAsync(T + (int64_t)i0 * n, p->d.Iout, (size_t)rows * n * sizeof(double),
                           hipMemcpyDeviceToDevice, p->stream) != hipSuccess)
            st = XBAR_ERR_DEVICE;
    }
    p->timing = timing;
    return st;
}

// T from the factorization by block recurrences.  The condensed system A is
// symmetric, so row i of T is g_sense W_i c_i with W_i the transpose of block row i
// of Y = A^-1 E (E: identity blocks at the last row; c_i: the condensed source
// coupling of row i, whose input vector is V_i c_i).  Y follows from the twisted
// factorization exactly as a sweep would with right-hand side E, on whole n_p x n_p
// blocks: the top chain's forward results are zero, so
//   bottom chain:  W_{m-1} = H_{m-1},  W_i = g W_{i+1} H_i       (i = m-2 .. kt+1)
//   twist:         W_kt = g W_{kt+1} H_kt                       (H_kt if kt = m-1)
//   back, up:      W_i = g W_{i+1} H_i                           (i = kt-1 .. 0)
//   back, down:    W_i = W_i + g W_{i-1} H_i                     (i = kt+1 .. m-1)
// (H_i symmetric, g = g_bl).  The two back chains share launches.
xbar_status transfer_by_blocks(xbar_plan p, double* T)
{
    const int m = p->g.m, n = p->g.n, n_p = p->n_p, kt = m / 2;
    const int64_t blk = (int64_t)n_p * n_p;
    double* W = reinterpret_cast<double*>(p->d.Z);
    const double* H = reinterpret_cast<const double*>(p->d.H);
    const double g = 1.0 / p->g.r_bl;
    auto Wb = [&](int i) { return W + i * blk; };
    auto Hb = [&](int i) { return H + i * blk; };
    auto one = [&](const double* A, const double* B, const double* C, double* out) {
        const XbkFrgJob j{A, B, C, out};
        return xbk_launch_frg_products(&j, 1, n_p, g, p->stream) == hipSuccess;
    };
    const size_t bytes = (size_t)blk * sizeof(double);
    if (kt + 1 < m) {
        if (hipMemcpyAsync(Wb(m - 1), Hb(m - 1), bytes, hipMemcpyDeviceToDevice, p->stream) != hipSuccess)
            return XBAR_ERR_DEVICE;
        for (int i = m - 2; i >= kt; --i)
            if (!one(Wb(i + 1), Hb(i), nullptr, Wb(i))) return XBAR_ERR_DEVICE;
    } else if (hipMemcpyAsync(Wb(kt), Hb(kt), bytes, hipMemcpyDeviceToDevice, p->stream) != hipSuccess) {
        return XBAR_ERR_DEVICE;
    }
    for (int s = 0;; ++s) {
        const int up = kt - 1 - s, down = kt + 1 + s;
        XbkFrgJob jobs[2];
        int nj = 0;
        if (up >= 0) jobs[nj++] = XbkFrgJob{Wb(up + 1), Hb(up), nullptr, Wb(up)};
        if (down < m) jobs[nj++] = XbkFrgJob{Wb(down - 1), Hb(down), Wb(down), Wb(down)};
        if (nj == 0) break;
        if (xbk_launch_frg_products(jobs, nj, n_p, g, p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
    }
    if (xbk_launch_transfer_rows(m, n, n_p, W, p->d.c, 1.0 / p->g.r_sense, T, p->stream) != hipSuccess)
        return XBAR_ERR_DEVICE;
    return XBAR_OK;
}

}  // namespace

extern "C" {

xbar_status xbar_set_factor_method(xbar_plan p, xbar_factor_method method)
{
    if (p == nullptr) return XBAR_ERR_ARG;
    if (method != XBAR_FACTOR_AUTO && method != XBAR_FACTOR_GJ && method != XBAR_FACTOR_NS &&
        method != XBAR_FACTOR_CHECKED)
        return XBAR_ERR_ARG;
    p->factor_method = method;
    return XBAR_OK;
}

xbar_status xbar_factor(xbar_plan p)
{
    if (p == nullptr) return XBAR_ERR_ARG;
    if (p->state != kAssembled) return XBAR_ERR_STATE;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    if (p->timing && !p->t_factor.begin(p->stream)) return XBAR_ERR_DEVICE;
    if (p->factor_method == XBAR_FACTOR_GJ) {
        p->ns_async = false;
        p->ns_used_host = 0;
        for (int& c : p->ns_launched) c = 0;
        if (launch_gj(p) != hipSuccess) return XBAR_ERR_DEVICE;
    } else {
        // AUTO reads the schedule back (and learns its launch counts) until it has
        // counts from an earlier factorization of this plan; then it runs asynchronously
        const bool checked = p->factor_method != XBAR_FACTOR_AUTO || !p->ns_hint_valid;
        p->ns_async = !checked;
        bool failed = false;
        if (run_ns(p, checked, &failed) != hipSuccess) return XBAR_ERR_DEVICE;
        if (failed && p->factor_method == XBAR_FACTOR_CHECKED) {
            // Redo the factorization by Gauss-Jordan elimination: rebuild E from the
            // plan's copy of G (the Newton-Schulz pass consumed part of it).
            hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, p->stream, p->d.flags,
                               (int)xbk::kNsFail);
            if (condense(p, p->d.Gc) != hipSuccess) return XBAR_ERR_DEVICE;
            if (launch_gj(p) != hipSuccess) return XBAR_ERR_DEVICE;
            p->gj_fallbacks++;
            for (int& h : p->ns_slots_hint) h = 0;
            p->ns_hint_valid = false;
        } else if (failed) {
            // Newton-Schulz only: report the miss through the sticky flags
            hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, p->stream, p->d.flags,
                               (int)xbk::kErrConv);
        }
    }
    if (p->prec == XBAR_BF16_IR || p->prec == XBAR_BF16_GMRES_IR) {
        // the trial's factor: the float32 inverse blocks at bfloat16 precision
        const int64_t count = (int64_t)p->g.m * p->n_p * p->n_p;
        hipLaunchKernelGGL(round_bf16_kernel, dim3(2048), dim3(256), 0, p->stream, reinterpret_cast<float*>(p->d.H),
                           count);
        if (hipGetLastError() != hipSuccess) return XBAR_ERR_DEVICE;
    }
    if (p->timing && !p->t_factor.end(p->stream)) return XBAR_ERR_DEVICE;
    p->state = kFactored;
    return XBAR_OK;
}

// Restarted flexible GMRES refinement of the condensed system (the kernels and the
// method are described in gmres.hip): u_0 = M^-1 V c, then up to ir_max_iter outer
// steps of k = kGmRestart Arnoldi steps each, with classical Gram-Schmidt applied
// twice; every launch is queued without a host read-back.
static_assert(xbk::kGmRestart == XBAR_GMRES_RESTART, "restart length of the header");

xbar_status gmres_solve(xbar_plan p, xbk::SweepArgs s, xbk::ResidualArgs r, int B)
{
    Buffers& d = p->d;
    constexpr int K = xbk::kGmRestart;
    const int nslab = (B + 15) / 16, Bp = 16 * nslab, m = p->g.m;
    xbk::GmPanel g{};
    g.m = m;
    g.n_p = p->n_p;
    g.nslab = nslab;
    const int want = std::max(1, 1024 / nslab);
    g.nchunk = std::min(m, want);
    g.rows_per_chunk = (m + g.nchunk - 1) / g.nchunk;
    g.nchunk = (m + g.rows_per_chunk - 1) / g.rows_per_chunk;
    g.P = (int64_t)nslab * m * 16 * p->n_p;
    g.slab_done = d.slab_done;
    g.slab_final = d.slab_final;
    const int64_t P = g.P;
    auto ok = [](hipError_t e) { return e == hipSuccess; };
    auto sweep = [&](int iter, const double* uin, double* uout) {
        s.iter = iter;
        s.Uin = uin;
        s.Uout = uout;
        if (p->timing && !p->t_ir_sweep.begin(p->stream)) return false;
        if (!ok(xbk_launch_sweep_ir(s, p->stream))) return false;
        return !p->timing || p->t_ir_sweep.end(p->stream);
    };
    auto resid = [&](const double* u, double* out, int matvec) {
        r.U = u;
        r.Rd = out;
        r.matvec = matvec;
        if (p->timing && !p->t_residual.begin(p->stream)) return false;
        if (!ok(xbk_launch_residual(r, p->stream))) return false;
        return !p->timing || p->t_residual.end(p->stream);
    };
    s.max_iter = 1 << 20;
    s.tol = -1.0;                        // the sweeps only apply the factor
    s.R = d.R;
    double* U = d.U[0];
    if (!sweep(0, d.gm_zero, U)) return XBAR_ERR_DEVICE;
    for (int it = 0; it < p->ir_max_iter; ++it) {
        double* V0 = d.gm_V;
        if (!resid(U, V0, 0)) return XBAR_ERR_DEVICE;
        if (!ok(xbk_gm_dots(g, V0, 1, V0, d.gm_part, d.gm_beta, Bp, false, true, p->stream)) ||
            !ok(xbk_gm_scale(g, V0, d.gm_beta, V0, reinterpret_cast<float*>(d.R), p->stream)) ||
            !ok(xbk_gm_fill(d.gm_H, (int64_t)(K + 1) * K * Bp, 0.0, p->stream)))
            return XBAR_ERR_DEVICE;
        for (int j = 0; j < K; ++j) {
            double* Zj = d.gm_Z + j * P;
            double* W = d.gm_V + (j + 1) * P;
            double* Hcol = d.gm_H + (int64_t)j * Bp;             // H[i][j] at Hcol + i K Bp
            if (!sweep(1, d.gm_zero, Zj) || !resid(Zj, W, 1)) return XBAR_ERR_DEVICE;
            for (int pass = 0; pass < 2; ++pass) {
                if (!ok(xbk_gm_dots(g, d.gm_V, j + 1, W, d.gm_part, d.gm_coef, Bp, false, false, p->stream)) ||
                    !ok(xbk_gm_axpy(g, d.gm_V, j + 1, d.gm_coef, Bp, W, p->stream)) ||
                    !ok(xbk_gm_add(g, j + 1, d.gm_coef, Bp, Hcol, K * Bp, p->stream)))
                    return XBAR_ERR_DEVICE;
            }
            double* hsub = Hcol + (int64_t)(j + 1) * K * Bp;
            if (!ok(xbk_gm_dots(g, W, 1, W, d.gm_part, hsub, Bp, false, true, p->stream)) ||
                !ok(xbk_gm_scale(g, W, hsub, W, j + 1 < K ? reinterpret_cast<float*>(d.R) : nullptr, p->stream)))
                return XBAR_ERR_DEVICE;
        }
        if (!ok(xbk_gm_lsq(g, d.gm_H, d.gm_beta, d.gm_y, p->stream)) ||
            !ok(xbk_gm_update(g, d.gm_Z, d.gm_y, U, d.gm_part, B, p->ir_tol, it, it + 1 == p->ir_max_iter,
                              d.flags, p->stream)))
            return XBAR_ERR_DEVICE;
    }
    if (!ok(xbk_gm_currents(g, B, p->g.n, 1.0 / p->g.r_sense, U, d.Iout, p->stream))) return XBAR_ERR_DEVICE;
    return XBAR_OK;
}

xbar_status xbar_solve_batch(xbar_plan p, const double* V, int32_t B, double* node_v)
{
    if (p == nullptr || V == nullptr) return XBAR_ERR_ARG;
    if (B < 1 || B > p->max_batch) return XBAR_ERR_ARG;
    if (p->state < kFactored) return XBAR_ERR_STATE;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    const int nslab = (B + 15) / 16;
    xbk::SweepArgs s{};
    s.m = p->g.m;
    s.n = p->g.n;
    s.n_p = p->n_p;
    s.B = B;
    s.nslab = nslab;
    s.g_bl = 1.0 / p->g.r_bl;
    s.g_sense = 1.0 / p->g.r_sense;
    s.H = p->d.H;
    s.c = p->d.c;
    s.V = V;
    s.Z = p->d.Z;
    s.Iout = p->d.Iout;
    s.flags = p->d.flags;
    s.sink = p->d.sink;
    const bool ir = p->prec != XBAR_FP64;
    // reciprocal ordering: the inputs drive the terminations, and the node voltages are
    // always recovered (into the plan's buffer) for the given crossbar's currents
    double* nv_solve = p->rev ? p->d.nv_rev : node_v;
    s.term = p->rev ? 1 : 0;
    s.node_v = ir ? nullptr : nv_solve;   // float64: recovery fused into the back sweep
    s.Gc = p->d.Gc;
    s.fr = p->d.fr;
    s.ip = p->d.ip;
    s.g_src = 1.0 / p->g.r_src;
    s.g_wl = 1.0 / p->g.r_wl;
    if (p->timing && !p->t_sweep.begin(p->stream)) return XBAR_ERR_DEVICE;
    if (!ir) {
        if (xbk_launch_sweep(s, p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
    } else {
        // float sweeps refined in float64: sweep 0 solves with V c, each later sweep
        // corrects U by the solution for the float64 residual of the previous U.
        hipLaunchKernelGGL(clear_slabs_kernel, dim3((16 * nslab + 255) / 256), dim3(256), 0, p->stream,
                           p->d.slab_done, p->d.dnorm, nslab);
        s.max_iter = 1 + p->ir_max_iter;
        s.tol = p->ir_tol;
        s.R = p->d.R;
        s.dnorm = p->d.dnorm;
        s.slab_done = p->d.slab_done;
        s.slab_final = p->d.slab_final;
        xbk::ResidualArgs r{};
        r.m = p->g.m;
        r.n = p->g.n;
        r.n_p = p->n_p;
        r.B = B;
        r.nslab = nslab;
        r.g_bl = 1.0 / p->g.r_bl;
        r.g_wl = 1.0 / p->g.r_wl;
        r.V = V;
        r.c = p->d.c;
        r.fr = p->d.fr;
        r.ip = p->d.ip;
        r.q = p->d.q;
        r.Gc = p->d.Gc;
        r.R = p->d.R;
        r.slab_done = p->d.slab_done;
        r.term = s.term;
        r.g_sense = 1.0 / p->g.r_sense;
        if (p->prec == XBAR_BF16_GMRES_IR) {
            const xbar_status gs = gmres_solve(p, s, r, B);
            if (gs != XBAR_OK) return gs;
            s.max_iter = 0;                  // the loop below is the classical refinement
        }
        for (int it = 0; it < s.max_iter; ++it) {
            s.iter = it;
            s.Uin = p->d.U[it & 1];
            s.Uout = p->d.U[(it + 1) & 1];
            if (it > 0) {
                r.U = p->d.U[it & 1];
                if (p->timing && !p->t_residual.begin(p->stream)) return XBAR_ERR_DEVICE;
                if (xbk_launch_residual(r, p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
                if (p->timing && !p->t_residual.end(p->stream)) return XBAR_ERR_DEVICE;
            }
            if (p->timing && !p->t_ir_sweep.begin(p->stream)) return XBAR_ERR_DEVICE;
            if (xbk_launch_sweep_ir(s, p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
            if (p->timing && !p->t_ir_sweep.end(p->stream)) return XBAR_ERR_DEVICE;
        }
    }
    if (p->timing && !p->t_sweep.end(p->stream)) return XBAR_ERR_DEVICE;
    if (nv_solve != nullptr && ir) {
        xbk::RecoverArgs r{};
        r.m = p->g.m;
        r.n = p->g.n;
        r.n_p = p->n_p;
        r.B = B;
        r.nslab = nslab;
        r.g_src = 1.0 / p->g.r_src;
        r.g_wl = 1.0 / p->g.r_wl;
        r.V = V;
        r.U[0] = p->d.U[0];
        r.U[1] = p->d.U[1];
        r.slab_final = p->d.slab_final;
        r.fr = p->d.fr;
        r.ip = p->d.ip;
        r.Gc = p->d.Gc;
        r.node_v = nv_solve;
        r.term = s.term;
        if (p->timing && !p->t_recover.begin(p->stream)) return XBAR_ERR_DEVICE;
        if (xbk_launch_recover(r, p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
        if (p->timing && !p->t_recover.end(p->stream)) return XBAR_ERR_DEVICE;
    }
    if (p->rev) {
        // the given crossbar's currents (and node voltages) from the reciprocal's
        hipLaunchKernelGGL(rev_outputs_kernel, dim3(grid_for((int64_t)B * p->og.m * p->og.n)), dim3(256), 0,
                           p->stream, p->d.nv_rev, B, p->og.m, p->og.n, 1.0 / p->og.r_sense, p->d.Iout, node_v);
        if (hipGetLastError() != hipSuccess) return XBAR_ERR_DEVICE;
    }
    p->backerr_valid = false;
    if (p->diagnostics && node_v != nullptr && p->og.n <= xbk_backward_error_max_n()) {
        // on the crossbar as given (reciprocal ordering: its conductances read through
        // the reciprocal's array)
        xbk::BackErrArgs be{};
        be.m = p->og.m;
        be.n = p->og.n;
        be.B = B;
        be.g_wl = 1.0 / p->og.r_wl;
        be.g_bl = 1.0 / p->og.r_bl;
        be.g_src = 1.0 / p->og.r_src;
        be.g_sense = 1.0 / p->og.r_sense;
        be.rev = p->rev ? 1 : 0;
        be.G = p->d.Gc;
        be.V = V;
        be.node_v = node_v;
        be.diag = p->d.diag;
        if (xbk_launch_reset_diag(p->d.diag, 2, p->stream) != hipSuccess ||
            xbk_launch_backward_error(be, p->stream) != hipSuccess)
            return XBAR_ERR_DEVICE;
        p->backerr_valid = true;
    }
    p->state = kSolved;
    p->last_B = B;
    return XBAR_OK;
}

xbar_status xbar_currents(xbar_plan p, double* I)
{
    if (p == nullptr || I == nullptr) return XBAR_ERR_ARG;
    if (p->state != kSolved) return XBAR_ERR_STATE;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    const size_t bytes = (size_t)p->last_B * p->og.n * sizeof(double);
    if (hipMemcpyAsync(I, p->d.Iout, bytes, hipMemcpyDeviceToDevice, p->stream) != hipSuccess)
        return XBAR_ERR_DEVICE;
    return XBAR_OK;
}

xbar_status xbar_transfer(xbar_plan p, double* T)
{
    if (p == nullptr || T == nullptr) return XBAR_ERR_ARG;
    if (p->state < kFactored) return XBAR_ERR_STATE;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    const xbar_status st = transfer_blocks_fit(p) ? transfer_by_blocks(p, T) : transfer_by_unit_solves(p, T);
    // the batch workspace no longer holds a caller's batch
    p->state = kFactored;
    p->last_B = 0;
    return st;
}

xbar_status xbar_transfer_apply(xbar_plan p, const double* T, const double* V, int32_t B, double* I)
{
    if (p == nullptr || T == nullptr || V == nullptr || I == nullptr || B < 1) return XBAR_ERR_ARG;
    const int64_t m = p->og.m, n = p->og.n;
    const int64_t i_bytes = (int64_t)B * n * 8;
    if (overlaps(I, i_bytes, V, (int64_t)B * m * 8) || overlaps(I, i_bytes, T, m * n * 8))
        return XBAR_ERR_ARG;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    if (xbk_launch_transfer_apply(B, (int)m, (int)n, V, T, I, p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
    return XBAR_OK;
}

xbar_status xbar_tiles_currents(const xbar_geometry* geom, int32_t T, int32_t B, const double* G, const double* V,
                                double* I, void* hip_stream)
{
    if (geom == nullptr || G == nullptr || V == nullptr || I == nullptr) return XBAR_ERR_ARG;
    const xbar_geometry g = *geom;
    if (g.m < 1 || g.n < 1 || g.n > XBAR_TILE_MAX_N || T < 1 || B < 1 || B > XBAR_TILE_MAX_B) return XBAR_ERR_ARG;
    if (!finite_pos(g.r_wl) || !finite_pos(g.r_bl) || !finite_pos(g.r_src) || !finite_pos(g.r_sense))
        return XBAR_ERR_ARG;
    const int64_t i_bytes = (int64_t)T * B * g.n * 8;
    if (overlaps(I, i_bytes, G, (int64_t)T * g.m * g.n * 8) || overlaps(I, i_bytes, V, (int64_t)T * B * g.m * 8))
        return XBAR_ERR_ARG;
    if (xbk_launch_tile_currents(T, g.m, g.n, B, 1.0 / g.r_wl, 1.0 / g.r_bl, 1.0 / g.r_src, 1.0 / g.r_sense, G, V, I,
                                 reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess) {
        (void)hipGetLastError();
        return XBAR_ERR_DEVICE;
    }
    return XBAR_OK;
}

xbar_status xbar_get_info(xbar_plan p, xbar_info* info)
{
    if (p == nullptr || info == nullptr) return XBAR_ERR_ARG;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    int flags[xbk::kNumFlags] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long diag[xbk::kNumDiag] = {0, 0, 0, 0};
    if (hipMemcpyAsync(flags, p->d.flags, sizeof(flags), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipMemcpyAsync(diag, p->d.diag, sizeof(diag), hipMemcpyDeviceToHost, p->stream) != hipSuccess)
        return XBAR_ERR_DEVICE;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return XBAR_ERR_DEVICE;
    std::memset(info, 0, sizeof(*info));
    info->state = p->state;
    info->last_batch = p->last_B;
    info->ir_iters = flags[xbk::kIrIters];
    info->workspace_bytes = p->bytes;
    info->block = p->n_p;
    // smallest pivot: decode the order-preserving key (+inf: no factorization yet)
    const unsigned long long k = diag[xbk::kDiagMinPivot];
    unsigned long long bits;
    if (k == 0ull) bits = 0x7FF8000000000000ull;
    else if (k >> 63) bits = k & 0x7FFFFFFFFFFFFFFFull;
    else bits = ~k;
    std::memcpy(&info->min_pivot, &bits, sizeof(double));
    if (p->backerr_valid) std::memcpy(&info->max_backward_err, &diag[xbk::kDiagBackErr], sizeof(double));
    else info->max_backward_err = -1.0;
    if (p->ns_async) {
        // what the asynchronous factorization needed becomes the next one's budget base
        info->factor_slots_used = flags[xbk::kNsUsed] + flags[xbk::kNsUsed + 1] + flags[xbk::kNsUsed + 2];
        bool all = true;
        for (int c = 0; c < 3; ++c) {
            const int rows = c == 0 ? p->g.m / 2 : c == 1 ? std::max(0, p->g.m - 1 - p->g.m / 2) : 1;
            all &= rows == 0 || flags[xbk::kNsUsed + c] > 0;
        }
        if (all) {
            for (int c = 0; c < 3; ++c) p->ns_slots_hint[c] = flags[xbk::kNsUsed + c];
        } else {
            p->ns_hint_valid = false;       // a budget ran out: the next factorization re-learns
        }
    } else {
        info->factor_slots_used = p->ns_used_host;
    }
    info->factor_slots_launched = p->ns_launched[0] + p->ns_launched[1] + p->ns_launched[2];
    xbar_status st = XBAR_OK;
    if (flags[xbk::kErrInput]) st = XBAR_ERR_INPUT;
    else if (flags[xbk::kErrPivot]) st = XBAR_ERR_NOT_SPD;
    else if (flags[xbk::kErrConv]) st = XBAR_ERR_NO_CONVERGENCE;
    info->device_error = (int32_t)st;
    return st;
}

xbar_status xbar_set_diagnostics(xbar_plan p, int32_t enable)
{
    if (p == nullptr) return XBAR_ERR_ARG;
    p->diagnostics = enable != 0;
    return XBAR_OK;
}

xbar_status xbar_debug_shift_pivots(xbar_plan p, double shift)
{
    if (p == nullptr || !std::isfinite(shift)) return XBAR_ERR_ARG;
    p->pivot_shift = shift;
    return XBAR_OK;
}

xbar_status xbar_set_timing(xbar_plan p, int32_t enable)
{
    if (p == nullptr) return XBAR_ERR_ARG;
    p->timing = enable != 0;
    return XBAR_OK;
}

xbar_status xbar_get_timing(xbar_plan p, xbar_timing* out, int32_t reset)
{
    if (p == nullptr || out == nullptr) return XBAR_ERR_ARG;
    if (!set_device(p)) return XBAR_ERR_DEVICE;
    PhaseTimer* all[] = {&p->t_condense, &p->t_factor, &p->t_sweep, &p->t_recover, &p->t_ir_sweep, &p->t_residual};
    for (PhaseTimer* t : all)
        if (!t->flush()) return XBAR_ERR_DEVICE;
    out->condense_ms = p->t_condense.ms;
    out->condense_launches = p->t_condense.launches;
    out->factor_ms = p->t_factor.ms;
    out->factor_launches = p->t_factor.launches;
    out->sweep_ms = p->t_sweep.ms;
    out->sweep_launches = p->t_sweep.launches;
    out->recover_ms = p->t_recover.ms;
    out->recover_launches = p->t_recover.launches;
    out->ir_sweep_ms = p->t_ir_sweep.ms;
    out->ir_sweep_launches = p->t_ir_sweep.launches;
    out->residual_ms = p->t_residual.ms;
    out->residual_launches = p->t_residual.launches;
    if (reset)
        for (PhaseTimer* t : all) {
            t->ms = 0.0;
            t->launches = 0;
        }
    return XBAR_OK;
}

xbar_status xbar_destroy(xbar_plan p)
{
    if (p == nullptr) return XBAR_OK;
    (void)set_device(p);
    (void)hipStreamSynchronize(p->stream);
    PhaseTimer* all[] = {&p->t_condense, &p->t_factor, &p->t_sweep, &p->t_recover, &p->t_ir_sweep, &p->t_residual};
    for (PhaseTimer* t : all) t->destroy();
    if (p->side) (void)hipStreamSynchronize(p->side);
    destroy_side(p);
    free_all(p);
    delete p;
    return XBAR_OK;
}

}  // extern "C"

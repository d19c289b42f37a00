/*
 * xbar.h - C ABI of the MI355X (gfx950) crossbar nodal solver.
 *
 * Problem (Kolinko et al., "XbarSim", Sec. II): an m x n memristive
 * crossbar with a linear device of conductance G[i][j] at every crosspoint,
 * a wire resistor between adjacent devices on every word line (WL, row i)
 * and bit line (BL, column j), a voltage source V_i driving each word line
 * and an output current through the termination of each bit line.  Nodal
 * analysis gives 2mn unknown node voltages and a symmetric system G v = I
 * (Sec. II.A, Eqs. 1-7), which the paper solves by LU decomposition once
 * per conductance map followed by forward and back substitution for every
 * input vector of a batch (Sec. II.C, Sec. III.A and III.D).
 *
 * This library orders the unknowns by crossbar row, so the system has m
 * diagonal blocks of 2n unknowns; it eliminates each row's word-line nodes
 * in closed form and runs a block LU (block-Thomas) over the rows on the
 * GPU.  The result is the same solution vector; see each call for what it
 * computes.
 *
 * Conventions
 *  - All pointers named "device" are device (HBM) pointers on the device
 *    that was current when the plan was created; the caller owns them.
 *  - All public floating-point data is float64, whatever the precision mode.
 *  - Node voltages use the paper's interleaved order (Sec. II.B):
 *      k = 2*(i*n + j) + s, s = 0 for WL(i,j), s = 1 for BL(i,j), 0-based.
 *  - Calls are asynchronous on the plan's HIP stream unless stated.
 *  - Errors found on the host are returned at once and touch no device
 *    state.  Errors found by kernels (bad conductance values, a pivot that
 *    is not positive, refinement that does not converge) set sticky device
 *    flags that xbar_get_info() reads (it synchronises the stream).
 *  - One host thread per plan.  Separate plans may share a device.
 */
#ifndef XBAR_H
#define XBAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xbar_plan_s* xbar_plan;          /* opaque, owned by the library */

typedef enum {
    XBAR_OK = 0,
    XBAR_ERR_ARG = 1,            /* invalid argument (host check)                      */
    XBAR_ERR_ALLOC = 2,          /* device memory allocation failed                    */
    XBAR_ERR_STATE = 3,          /* call out of order (see xbar_factor / solve_batch) */
    XBAR_ERR_NOT_SPD = 4,        /* a block pivot was not positive and finite          */
    XBAR_ERR_NO_CONVERGENCE = 5, /* iterative refinement missed its tolerance          */
    XBAR_ERR_DEVICE = 6,         /* no usable device, or a HIP runtime error           */
    XBAR_ERR_INPUT = 7           /* conductances not finite and positive (device check)*/
} xbar_status;

typedef enum {
    XBAR_FP64 = 0,      /* factor and substitution in float64 (the paper's method)         */
    XBAR_FP32_IR = 1,   /* factor and substitution in float32 on MFMA, refined in float64  */
    XBAR_BF16_IR = 2,   /* trial: as XBAR_FP32_IR, with the factor's inverse blocks rounded
                           to bfloat16 values (8-bit significand, ties to even) before the
                           float32 sweeps; measures whether a bfloat16-accurate factor still
                           drives the float64 refinement (else XBAR_ERR_NO_CONVERGENCE) */
    XBAR_BF16_GMRES_IR = 3 /* the XBAR_BF16_IR factor used as the preconditioner of a
                           restarted flexible GMRES in float64 (GMRES-based iterative
                           refinement, Carson and Higham): u_0 = M^-1 V c, then per outer
                           step the float64 residual, XBAR_GMRES_RESTART Arnoldi steps on
                           A M^-1 (M^-1: one float32 sweep of the factor; classical
                           Gram-Schmidt applied twice), the least-squares solution, and the
                           correction d.  A slab of input vectors stops when every vector's
                           max |d| <= ir_tol max |u|; ir_max_iter counts outer steps, and
                           ir_iters reports them.  Needs 2 XBAR_GMRES_RESTART + 4 float64
                           panels of ceil(max_batch / 16) m 16 n_p values.              */
} xbar_precision;

#define XBAR_GMRES_RESTART 8

typedef struct {
    int32_t m;          /* word lines (rows),   1 <= m                                  */
    int32_t n;          /* bit lines (columns), 1 <= n <= XBAR_MAX_N                     */
    double r_wl;        /* word-line segment resistance, ohm, finite > 0 (Sec. II.A)    */
    double r_bl;        /* bit-line segment resistance, ohm, finite > 0                 */
    double r_src;       /* resistance from source V_i to WL(i,0), ohm, finite > 0.
                           Eq. 5 puts a word-line segment there: the paper's model is
                           r_src = r_wl.                                                */
    double r_sense;     /* termination from BL(m-1,j) to 0 V, ohm, finite > 0.  The
                           paper's model terminates with a bit-line segment,
                           r_sense = r_bl.                                              */
} xbar_geometry;

#define XBAR_MAX_N 512

typedef struct {
    int32_t state;              /* 0 created, 1 assembled, 2 factored, 3 solved               */
    int32_t last_batch;         /* B of the last xbar_solve_batch                             */
    int32_t ir_iters;           /* refinement steps taken by the slowest input slab (IR modes)*/
    int32_t device_error;       /* sticky xbar_status found on the device, 0 if none          */
    int64_t workspace_bytes;    /* device memory held by the plan                             */
    int32_t block;              /* padded block size used for the row blocks                  */
    int32_t reserved;
    double min_pivot;           /* smallest pivot the last factorization met (Sec. II.C: the
                                   LU's pivots): the smallest diagonal entry of any block
                                   pivot for Newton-Schulz, the smallest scalar pivot for the
                                   Gauss-Jordan elimination; +inf before a factorization.
                                   Not positive => XBAR_ERR_NOT_SPD.                           */
    double max_backward_err;    /* largest normwise backward error ||b - A v||_inf /
                                   (||A||_inf ||v||_inf + ||b||_inf) over the last batch's
                                   node voltages v for the nodal system A v = b of Sec. II.A
                                   (Eqs. 5-7), when xbar_set_diagnostics is on and the batch
                                   wrote node voltages; -1 when not measured                  */
    int32_t factor_slots_used;  /* Newton-Schulz launches the last factorization needed       */
    int32_t factor_slots_launched; /* launches it queued (the asynchronous budget)           */
} xbar_info;

/*
 * Create a plan for one crossbar geometry.  Validates the geometry and the
 * options on the host, then allocates all device workspace for batches of
 * up to max_batch input vectors (nothing is allocated by later calls).
 *   p            precision mode.
 *   max_batch    1 <= max_batch.
 *   ir_tol       IR modes: a slab of input vectors stops refining when, for each
 *                of its vectors, the error estimate |d| min(1, |d| / |d_prev|)
 *                (d: the latest correction of the bit-line voltages, max norm)
 *                is <= ir_tol times the largest bit-line voltage; 0 selects
 *                1e-12.  This bounds the forward error of the solution (the
 *                estimate of a contracting iteration), not its backward error;
 *                xbar_set_diagnostics measures the latter after the solve.
 *                Must be finite, 0 <= ir_tol < 1.  Ignored for FP64.
 *   ir_max_iter  IR modes: refinement steps allowed, 1..100 (0 selects 10).
 *   hip_stream   hipStream_t the plan's work is queued on (NULL = null stream).
 *                The plan also creates one stream of its own (default priority,
 *                non-blocking), used only inside xbar_factor and joined back to
 *                hip_stream before that call returns; xbar_destroy releases it.
 * Returns XBAR_ERR_ARG, XBAR_ERR_DEVICE, XBAR_ERR_ALLOC or XBAR_OK.
 */
xbar_status xbar_create(const xbar_geometry* geom, xbar_precision p, int32_t max_batch,
                        double ir_tol, int32_t ir_max_iter, void* hip_stream, xbar_plan* out);

/*
 * Order of the block rows (Sec. III.B: the matrix bandwidth follows the side the
 * nodes are numbered along).  ROWS: one row block per word line, of size n (the
 * ordering of Sec. II.B; needs n <= XBAR_MAX_N).  SMALLER: row blocks of size
 * min(m, n); when n > m the plan solves the reciprocal crossbar, turned by 180
 * degrees and transposed (word and bit lines exchanged, r_src and r_sense
 * exchanged), whose inputs drive its bit-line terminations; currents, node voltages
 * (in the given crossbar's order), the transfer matrix and the backward error are
 * those of the crossbar as given.  That plan always recovers the node voltages (the
 * given crossbar's currents come from them) and holds a buffer of max_batch 2 m n
 * doubles for them.  AUTO: ROWS when n <= m; when n > m, SMALLER if n > XBAR_MAX_N,
 * else whichever of the two a cost model of the factor, measured on gfx950, finds
 * faster (the shorter chain of row blocks wins unless the blocks are large).
 */
typedef enum { XBAR_ORDER_AUTO = 0, XBAR_ORDER_ROWS = 1, XBAR_ORDER_SMALLER = 2 } xbar_ordering;

/*
 * xbar_create with an ordering (xbar_create is this with XBAR_ORDER_AUTO).  Returns
 * XBAR_ERR_ARG also for an unknown ordering and for ROWS with n > XBAR_MAX_N.
 * xbar_get_info's block field reports the padded row-block size the plan uses.
 */
xbar_status xbar_create_ordered(const xbar_geometry* geom, xbar_precision p, int32_t max_batch,
                                double ir_tol, int32_t ir_max_iter, void* hip_stream, int32_t ordering,
                                xbar_plan* out);

/*
 * Assemble the nodal equations (Sec. II.A-II.B, Eqs. 1-7) for the device
 * conductances G: device pointer, [m][n] row-major, siemens, each finite and
 * > 0 (a value that is not sets XBAR_ERR_INPUT on the device).  The library
 * copies what it needs; G may be reused after the call is queued and the
 * stream has passed it.  Invalidates any previous factorization.
 */
xbar_status xbar_assemble(xbar_plan plan, const double* G);

/*
 * LU-decompose the assembled system once per conductance map (Sec. II.C):
 * a block LU over the m row blocks.  Requires a prior xbar_assemble
 * (otherwise XBAR_ERR_STATE).  A pivot that is not positive sets
 * XBAR_ERR_NOT_SPD on the device (see xbar_info.min_pivot).  In the default
 * method (XBAR_FACTOR_AUTO) every factorization of a plan after its first is
 * asynchronous and reads nothing back, so it can be captured into a HIP graph
 * with the other calls: the plan's own second stream is forked from and joined
 * back to the plan stream by events within the call.  See
 * xbar_set_factor_method for the details and the other methods.
 */
xbar_status xbar_factor(xbar_plan plan);

/*
 * Forward and back substitution for a batch of input vectors (Sec. II.C,
 * batch mode of Sec. III.A/III.D), reusing the factorization.
 *   V       device, [B][m] row-major, volts (input vector b drives WL i with V[b][i]).
 *   B       1 <= B <= max_batch.
 *   node_v  device, [B][2mn] node voltages in the paper's order, or NULL to
 *           skip writing them (the output currents are still produced).
 * Requires a prior xbar_factor (XBAR_ERR_STATE otherwise).  Any number of
 * calls may follow one factorization.  IR modes run the refinement inside
 * this call; failing to converge sets XBAR_ERR_NO_CONVERGENCE on the device.
 */
xbar_status xbar_solve_batch(xbar_plan plan, const double* V, int32_t B, double* node_v);

/*
 * Output currents of the last solved batch: I[b][j] = V_BL(m-1, j) / r_sense,
 * the current through the termination of bit line j, amperes, positive into
 * the sense resistor (Sec. II).  I: device, [B][n] row-major.
 * Requires a prior xbar_solve_batch (XBAR_ERR_STATE otherwise).
 */
xbar_status xbar_currents(xbar_plan plan, double* I);

/*
 * Transfer matrix of the factored crossbar: T[i][j] = the output current of bit
 * line j (as xbar_currents reports it) when word line i is driven with 1 V and
 * every other source with 0 V.  The nodal system G v = I has a right-hand side
 * that is linear in the source voltages (Sec. II.A, Eqs. 5-7), so the currents
 * of any input vector are I[b][j] = sum_i V[b][i] T[i][j]: see
 * xbar_transfer_apply.  How T is computed from the plan's factorization:
 *  - XBAR_FP64 plans whose max_batch, rounded up to 16, is at least the padded
 *    block size (n rounded up to 64): by block recurrences.  The condensed
 *    system is symmetric, so row i of T is g_sense W_i c_i, with W_i the
 *    transposed block row i of the inverse applied to identity blocks at the
 *    last row; the W_i follow from the factorization by the substitution
 *    recurrences on whole blocks (about m dependent block products);
 *  - otherwise: by solving the m unit inputs, min(max_batch, m) of them per
 *    xbar_solve_batch, without node voltages, in the plan's precision mode.
 *   T  device, [m][n] row-major, amperes per volt; caller-owned.
 * Requires a prior xbar_factor (XBAR_ERR_STATE otherwise).  Uses the plan's
 * batch workspace: the result of an earlier xbar_solve_batch is dropped and
 * xbar_currents returns XBAR_ERR_STATE until the next xbar_solve_batch.  Not
 * counted by the phase timers.  Device errors (e.g. IR modes not converging)
 * set the sticky flags as xbar_solve_batch does.
 */
xbar_status xbar_transfer(xbar_plan plan, double* T);

/*
 * Output currents through the transfer matrix: I[b][j] = sum_i V[b][i] T[i][j],
 * a float64 matrix-core product queued on the plan's stream.  Exact up to
 * rounding for the linear network of Sec. II.A, and the same result as
 * xbar_solve_batch + xbar_currents for the conductances T was computed from.
 *   T  device, [m][n] row-major, from xbar_transfer (of this plan or another
 *      with the same m and n).
 *   V  device, [B][m] row-major, volts.
 *   B  1 <= B; not bounded by max_batch (the call uses no plan workspace).
 *   I  device, [B][n] row-major, amperes; must not overlap V or T.
 * Independent of the plan's state.  XBAR_ERR_ARG on NULL pointers, B < 1 or
 * overlapping I; XBAR_ERR_DEVICE on a launch error.
 */
xbar_status xbar_transfer_apply(xbar_plan plan, const double* T, const double* V, int32_t B, double* I);

/*
 * Output currents of T small crossbars of one shape, each with its own
 * conductances and input vectors, in one launch with one workgroup per
 * crossbar (the partitioned crossbars of Sec. III.C, solved by the method of
 * Sec. II.A-II.C: word-line elimination per row, block LU over the rows
 * top-down, forward substitution; the bottom row's forward result gives the
 * currents, so no back substitution is needed).  Needs no plan and allocates
 * nothing.
 *   geom   1 <= m, 1 <= n <= XBAR_TILE_MAX_N; resistances as for xbar_create.
 *   T      number of crossbars, >= 1.
 *   B      input vectors per crossbar, 1 <= B <= XBAR_TILE_MAX_B.
 *   G      device, [T][m][n] siemens.   V  device, [T][B][m] volts.
 *   I      device, [T][B][n] amperes, as xbar_currents; must not overlap G or V.
 *   hip_stream  hipStream_t the launch is queued on (NULL = null stream).
 * Asynchronous.  A crossbar with a conductance that is not finite and
 * positive gets NaN currents (the others are unaffected).  Returns
 * XBAR_ERR_ARG (host checks), XBAR_ERR_DEVICE (launch error) or XBAR_OK.
 */
#define XBAR_TILE_MAX_N 64
#define XBAR_TILE_MAX_B 256
xbar_status xbar_tiles_currents(const xbar_geometry* geom, int32_t T, int32_t B, const double* G, const double* V,
                                double* I, void* hip_stream);

/*
 * ---- Heterogeneous batches of crossbars ------------------------------------
 *
 * Many independent crossbars of mixed shapes (the partitioned crossbars of
 * Sec. III.C, each solved by the method of Sec. II.A-II.C), grouped by the caller
 * into classes of one shape: the output currents of every crossbar for its own
 * input vectors, in one call that queues every class's launches on a few streams
 * forked from, and joined back to, the caller's stream.  The call allocates
 * nothing and reads nothing back, so it can be captured into a HIP graph.
 *
 * How a class is solved (`method`, chosen per class, e.g. by a tuner):
 *   XBAR_TILE_ONE_WG    one workgroup per crossbar (n <= XBAR_TILE_MAX_N), the whole
 *                       solve in one launch, blocks padded to `block` (16, 32 or 64,
 *                       >= n; 0 picks the smallest); `split` (1..4) workgroups per
 *                       crossbar, each forward-substituting a share of its vectors
 *                       after redoing the factorization;
 *   XBAR_TILE_PIPELINE  the plan path's kernels batched over the class (n <=
 *                       XBAR_MAX_N): condensation, the twisted block Gauss-Jordan
 *                       factorization and the float64 currents-only sweep, each
 *                       covering every crossbar of the class per launch; `block`
 *                       and `split` must be 0 and 1.
 * `transpose` = 1 solves the class through its reciprocal problem instead, which
 * orders the row blocks by the smaller side when m < n: the network is reciprocal,
 * so the current into the sense resistor of bit line j per volt on word line i,
 * T[i][j], is the current into the source resistor of word line i per volt at the
 * sense terminal of bit line j (Sec. II.A's network with sources and sinks
 * exchanged).  That problem is the crossbar turned by a half turn and transposed
 * (n rows, m columns, word-line and bit-line segment resistances swapped, r_sense as
 * source and r_src as sense resistance) driven by the n unit inputs; `method`,
 * `block` and `split` apply to it (so they are checked against its n' = m columns
 * and n <= XBAR_TILE_MAX_B unit inputs), and I = V T follows by one product per
 * crossbar.
 * A crossbar with a conductance that is not finite and positive, or a pivot that
 * is not positive, gets NaN currents; the other crossbars are unaffected.
 */
#define XBAR_TILE_ONE_WG 0
#define XBAR_TILE_PIPELINE 1
typedef struct {
    int32_t m, n;       /* shape of the class's crossbars (rows, columns)             */
    int32_t count;      /* crossbars in the class, >= 1                                */
    int32_t B;          /* input vectors per crossbar, 1 .. XBAR_TILE_MAX_B            */
    int32_t method;     /* XBAR_TILE_ONE_WG or XBAR_TILE_PIPELINE                      */
    int32_t block;      /* XBAR_TILE_ONE_WG: padded block size, 0 = smallest           */
    int32_t split;      /* XBAR_TILE_ONE_WG: workgroups per crossbar (1..4)            */
    int32_t transpose;  /* 1: through the reciprocal problem (see above), else 0      */
} xbar_tile_class;

typedef struct xbar_tiles_s* xbar_tiles;    /* opaque, owned by the library */

/* Validate the classes and resistances (as xbar_create's) on the host, allocate the
 * pipeline classes' device workspace and `streams` (1..8) streams of default priority
 * with their events.  hip_stream: the caller's stream (NULL = null stream).  Returns
 * XBAR_ERR_ARG, XBAR_ERR_DEVICE, XBAR_ERR_ALLOC or XBAR_OK. */
xbar_status xbar_tiles_create(const xbar_tile_class* classes, int32_t nclasses, double r_wl, double r_bl,
                              double r_src, double r_sense, int32_t streams, void* hip_stream, xbar_tiles* out);

/* Output currents of every class: host arrays of nclasses device pointers, class k's
 * G[k] [count][m][n] siemens, V[k] [count][B][m] volts, I[k] [count][B][n] amperes
 * (as xbar_currents; must not overlap G[k] or V[k]).  Asynchronous on the caller's
 * stream; the pointers may change from call to call.  XBAR_ERR_ARG on a NULL
 * pointer, XBAR_ERR_DEVICE on a launch error. */
xbar_status xbar_tiles_run(xbar_tiles tiles, const double* const* G, const double* const* V, double* const* I);

/* Device bytes the batch holds (-1 for NULL). */
int64_t xbar_tiles_workspace_bytes(xbar_tiles tiles);

/* Synchronise the caller's stream and the batch's streams, then free everything.
 * NULL is a no-op. */
xbar_status xbar_tiles_destroy(xbar_tiles tiles);

/*
 * Synchronise the plan's stream and report its state.  Returns the sticky
 * device error (XBAR_ERR_INPUT, XBAR_ERR_NOT_SPD, XBAR_ERR_NO_CONVERGENCE)
 * if one was raised, XBAR_ERR_DEVICE on a HIP error, else XBAR_OK.
 * Reading the flags does not clear them; xbar_assemble does.
 */
xbar_status xbar_get_info(xbar_plan plan, xbar_info* info);

/*
 * How xbar_factor inverts the pivot blocks of the block LU.
 *   XBAR_FACTOR_AUTO (default): Newton-Schulz iteration on the matrix cores, on
 *       a schedule driven by the device.  The first factorization of a plan
 *       reads the schedule back (it synchronises the plan's stream) and so
 *       learns how many launches each of its three schedules needs; later ones
 *       are asynchronous and capturable: each schedule gets that many launches
 *       plus a margin of extra rounds (launches past a schedule's end do
 *       nothing), and nothing is read back.  xbar_get_info refreshes the
 *       counts from the device.  A block that misses its tolerance, or a budget
 *       that runs out, sets XBAR_ERR_NO_CONVERGENCE on the device (after a
 *       budget ran out the next factorization reads back again); the caller may
 *       then refactor, or use XBAR_FACTOR_CHECKED or XBAR_FACTOR_GJ.  To capture
 *       a plan's factorization into a graph, factor it once eagerly first.
 *   XBAR_FACTOR_GJ: blocked Gauss-Jordan elimination only (asynchronous).
 *   XBAR_FACTOR_NS: Newton-Schulz; the call reads the schedule states back and
 *       launches until every row has finished (it synchronises the plan's
 *       stream); a block that misses its tolerance sets XBAR_ERR_NO_CONVERGENCE.
 *   XBAR_FACTOR_CHECKED: as XBAR_FACTOR_NS, but a missed tolerance makes the
 *       call redo the factorization by Gauss-Jordan elimination.
 * Host-only; takes effect at the next xbar_factor.
 */
typedef enum { XBAR_FACTOR_AUTO = 0, XBAR_FACTOR_GJ = 1, XBAR_FACTOR_NS = 2, XBAR_FACTOR_CHECKED = 3 } xbar_factor_method;
xbar_status xbar_set_factor_method(xbar_plan plan, xbar_factor_method method);

/*
 * Solution diagnostics (host-only switch, off by default).  When on, every
 * xbar_solve_batch that writes node voltages also measures their normwise
 * backward error for the nodal system of Sec. II.A (one extra pass over the
 * node voltages, queued on the plan stream), reported as
 * xbar_info.max_backward_err.  Returns XBAR_ERR_ARG for a NULL plan.
 */
xbar_status xbar_set_diagnostics(xbar_plan plan, int32_t enable);

/*
 * Test hook, not for use in production: from the next xbar_assemble on,
 * subtract `shift` siemens from every diagonal entry of the condensed bit-line
 * blocks E_i before the factorization (0 switches it off).  Only the
 * factorization sees the shift; with a shift above the blocks' diagonal the
 * factor meets pivots that are not positive and reports XBAR_ERR_NOT_SPD, so
 * that path can be exercised with valid conductances.  XBAR_ERR_ARG for a NULL
 * plan or a shift that is not finite.
 */
xbar_status xbar_debug_shift_pivots(xbar_plan plan, double shift);

/*
 * Phase timing, measured with HIP events recorded on the plan's stream
 * around each phase of the calls above (only while enabled): one interval
 * per xbar_assemble (condense), per xbar_factor (all its kernels), per
 * xbar_solve_batch (its substitution sweeps; in FP64 mode that is exactly
 * one kernel, the sweep with the word-line recovery fused) and per
 * word-line recovery launch of the IR modes; inside the IR modes' solve,
 * also one interval per float32 sweep launch and per float64 residual
 * launch.  Times are accumulated milliseconds; *_launches count the
 * intervals.  Do not enable while capturing a graph.
 */
typedef struct {
    double condense_ms;   int64_t condense_launches;   /* xbar_assemble                 */
    double factor_ms;     int64_t factor_launches;     /* xbar_factor (all its kernels) */
    double sweep_ms;      int64_t sweep_launches;      /* substitution sweeps           */
    double recover_ms;    int64_t recover_launches;    /* word-line recovery + output   */
    double ir_sweep_ms;   int64_t ir_sweep_launches;   /* IR modes: each float32 sweep  */
    double residual_ms;   int64_t residual_launches;   /* IR modes: each float64 residual */
} xbar_timing;

/* Enable (1) or disable (0) per-kernel timing.  Host-only; never fails on a valid plan. */
xbar_status xbar_set_timing(xbar_plan plan, int32_t enable);

/* Synchronise, add up all timed launches so far into *out; reset != 0 clears them. */
xbar_status xbar_get_timing(xbar_plan plan, xbar_timing* out, int32_t reset);

/* Synchronise and free every device buffer of the plan.  NULL is a no-op. */
xbar_status xbar_destroy(xbar_plan plan);

/*
 * ---- Learned current surrogate ------------------------------------------
 *
 * A small convolutional network (an extension: the paper has no learned
 * part) predicts the relative parasitic correction of each bit-line current,
 * delta_j = (I_j - I0_j) / I0_j with I0 = G^T V, the currents of the same
 * crossbar without wire resistance (the zero-resistance limit of the nodal
 * equations of Sec. II.A).  Its training targets come from the exact solver
 * above, which stays the reference for its error.  These calls are the
 * network's steps; the caller owns every buffer (device memory, float32
 * activations [B][C][H][W] with H = m rows and W = n columns, weights
 * [O][C][3][3], biases [O]).  All convolutions are 3 x 3 cross-correlations
 * with zero padding of one crosspoint.  Each call checks its arguments on the
 * host (XBAR_ERR_ARG: a size out of range, a NULL pointer, an output that
 * overlaps an input), queues its kernels on `stream` and returns without
 * waiting; XBAR_ERR_DEVICE reports a failed launch.  Sizes: 1 <= B <= 65535,
 * H, W >= 1, 1 <= C, O <= XBAR_SG_MAX_CHANNELS.
 */
#define XBAR_SG_MAX_CHANNELS 32
#define XBAR_SG_FEATURES 7
#define XBAR_SG_MAX_LINE 2048

/* X [B][7][m][n] float32 from G [B][m][n] (S, > 0), V [B][m] (V), r [B] (ohm,
 * the segment resistance), m, n <= XBAR_SG_MAX_LINE: log10(G) + 5, 2 V_i,
 * (r - 3) / 2, the column and row positions 2 j / (n - 1) - 1 and
 * 2 i / (m - 1) - 1 (0 for n or m = 1), and the line totals that set the drops
 * at the line ends, 1e4 mean_j' G[i][j'] (row i) and 1e4 mean_i' G[i'][j] 2 V_i'
 * (column j). */
xbar_status xbar_sg_features(int32_t B, int32_t m, int32_t n, const double* G, const double* V, const double* r,
                             float* X, void* stream);

/* y[b][o][p][q] = bias[o] + sum_{c,dy,dx} w[o][c][dy][dx] x[b][c][p+dy-1][q+dx-1],
 * then max(y, 0) if relu != 0.  x [B][C][H][W], y [B][O][H][W]. */
xbar_status xbar_sg_conv_forward(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, int32_t relu,
                                 const float* x, const float* w, const float* bias, float* y, void* stream);

/* Input gradient of a convolution: with g = gy, multiplied by [ymask > 0] when
 * ymask (the layer's ReLU output, same shape as gy) is not NULL,
 * gx[b][c][p][q] = sum_{o,dy,dx} w[o][c][dy][dx] g[b][o][p-dy+1][q-dx+1], multiplied
 * by [xmask > 0] when xmask (the layer's input, the previous layer's ReLU output,
 * same shape as gx) is not NULL: then gx is the gradient before that ReLU. */
xbar_status xbar_sg_conv_backward_data(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* gy,
                                       const float* ymask, const float* w, const float* xmask, float* gx,
                                       void* stream);

/* Weight and bias gradients, g masked as above: gw[o][c][dy][dx] = sum_{b,p,q}
 * g[b][o][p][q] x[b][c][p+dy-1][q+dx-1], gb[o] = sum g[b][o][p][q].  work:
 * at least xbar_sg_workspace_floats(C, O) floats (partial sums, summed in a
 * fixed order, so the result is deterministic). */
xbar_status xbar_sg_conv_backward_weight(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* x,
                                         const float* gy, const float* ymask, float* gw, float* gb, float* work,
                                         int64_t work_floats, void* stream);

/* Floats of workspace xbar_sg_conv_backward_weight needs (-1 for bad C, O). */
int64_t xbar_sg_workspace_floats(int32_t C, int32_t O);

/* For callers that cannot allocate (code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc): xbar_sg_conv_backward_weight without the
 * workspace argument.  The partial sums go to a device array inside the library,
 * sized for the largest channel counts, xbar_sg_workspace_floats(32, 32) floats
 * (about 19 MB), which each GPU the library runs on holds from the first call on
 * that GPU until the process ends; the call allocates nothing (no hipMalloc, no
 * library allocation).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (concurrent streams, other host threads) race and must be
 * serialised by the caller.  Same result, bit for bit, as
 * xbar_sg_conv_backward_weight on the same inputs.  XBAR_ERR_ARG as that call
 * (sizes, NULL pointers, gw overlapping gb); XBAR_ERR_DEVICE when the array's
 * address cannot be obtained on the current device or a launch fails. */
xbar_status xbar_sg_conv_backward_weight_noalloc(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O,
                                                 const float* x, const float* gy, const float* ymask, float* gw,
                                                 float* gb, void* stream);

/* The same three convolutions on the bfloat16 matrix cores: each call has the
 * arguments, layouts and checks of its float32 counterpart above, and computes the
 * same sums with every operand rounded to bfloat16 (8-bit significand, nearest, ties
 * to even; activations, gradients and weights stay float32 in memory) and the
 * products accumulated in float32.  The input-gradient masks and the workspace are as
 * for the float32 calls (xbar_sg_workspace_floats). */
xbar_status xbar_sg_conv_forward_bf16(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, int32_t relu,
                                      const float* x, const float* w, const float* bias, float* y, void* stream);
xbar_status xbar_sg_conv_backward_data_bf16(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* gy,
                                            const float* ymask, const float* w, const float* xmask, float* gx,
                                            void* stream);
xbar_status xbar_sg_conv_backward_weight_bf16(int32_t B, int32_t H, int32_t W, int32_t C, int32_t O, const float* x,
                                              const float* gy, const float* ymask, float* gw, float* gb, float* work,
                                              int64_t work_floats, void* stream);

/* Column readouts and loss of the last map Y [B][2][m][n] (float32):
 * yhat_j = mean_i Y[b][0][i][j] (the correction), s_j = mean_i Y[b][1][i][j] (the
 * error estimate), e = yhat - delta (delta [B][n] float64), and the normalised log
 * squared error t = (log(e^2 + eps) - mu) / sigma (eps, mu, sigma = XBAR_SG_EST_EPS,
 * XBAR_SG_EST_MU, XBAR_SG_EST_SIGMA), held constant.  Loss mean(e^2) + lam
 * mean((s - t)^2): gY[b][0][i][j] = 2 e_j / (B n m), gY[b][1][i][j] = lam 2 (s_j - t_j)
 * / (B n m); err2 [B][2] = {sum_j e_j^2, sum_j (s_j - t_j)^2}.  lam >= 0.  (A caller
 * that keeps the estimate out of the shared layers zeroes gY[b][1] after the last
 * layer's weight gradient and before its input gradient.) */
#define XBAR_SG_EST_EPS 1e-8
#define XBAR_SG_EST_MU (-12.0)
#define XBAR_SG_EST_SIGMA 4.0
xbar_status xbar_sg_readout_loss(int32_t B, int32_t m, int32_t n, const float* Y, const double* delta, double lam,
                                 float* gY, double* err2, void* stream);

/* One Adam step (bias-corrected, step t >= 1) over count float32 parameters p
 * with gradients g and moments m1, m2, all updated in place. */
xbar_status xbar_sg_adam(int64_t count, float* p, const float* g, float* m1, float* m2, double lr, double b1,
                         double b2, double eps, int32_t t, void* stream);

/* Surrogate currents I [B][n] float64 = (G^T V)_j (1 + yhat_j), yhat_j = mean_i Y[b][0][i][j],
 * and, when est is not NULL, the predicted relative current error
 * est [B][n] = exp((sigma s_j + mu) / 2) / |1 + yhat_j|, s_j = mean_i Y[b][1][i][j]. */
xbar_status xbar_sg_predict(int32_t B, int32_t m, int32_t n, const float* Y, const double* G, const double* V,
                            double* I, double* est, void* stream);

/* Training targets delta [S][n] = (I - I0) / I0 elementwise (I: exact currents, I0 = G^T V,
 * both [S][n] float64 device arrays). */
xbar_status xbar_sg_targets(int32_t S, int32_t n, const double* I, const double* I0, double* delta, void* stream);

/* Calibration ratios ratio [B] of predictions Ip [B][n] with error estimates est [B][n]
 * against exact currents I [B][n]: max_j |Ip - I| / |I| over the columns with I != 0,
 * divided by max_j est; NaN for a sample with no such column, a maximum that is not
 * finite, or a non-positive estimate maximum.  The caller's quantile of the finite
 * ratios is the scale kappa of the estimate (split-conformal calibration). */
xbar_status xbar_sg_calib_ratios(int32_t B, int32_t n, const double* Ip, const double* I, const double* est,
                                 double* ratio, void* stream);

/* Routing of checked predictions: flag [B] int32 = 1 (solve exactly) unless
 * kappa max_j est[b][j] <= tol, every I[b][j] is finite, every G[b] entry is finite and
 * positive and every V[b] entry is finite; else 0.  G [B][m][n], V [B][m], I, est [B][n]. */
xbar_status xbar_sg_route(int32_t B, int32_t m, int32_t n, const double* G, const double* V, const double* I,
                          const double* est, double kappa, double tol, int32_t* flag, void* stream);

/* Static, NUL-terminated name of a status code. */
const char* xbar_status_string(xbar_status s);

#ifdef __cplusplus
}
#endif

#endif /* XBAR_H */

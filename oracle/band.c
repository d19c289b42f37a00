/*
 * Plain CPU reference kernels for the crossbar oracle (test infrastructure,
 * not part of the GPU library; nothing here is shared with it).
 *
 *  - band_lu:        Doolittle LU of a banded matrix without pivoting,
 *                    L unit lower and U upper, as in the paper's Sec. II.C
 *                    (G = LU, then Ly = I and UV = y).
 *  - band_solve:     forward substitution L y = b, then back substitution
 *                    U x = y, for many right-hand sides at once.
 *  - netlist_residual_ld: Kirchhoff current-law residual b - A x evaluated
 *                    from the resistor list in long double (x86 80-bit),
 *                    used for the oracle's iterative refinement.
 *
 * Band storage: row r holds columns c in [r-w, r+w] at ab[r*(2w+1) + c-r+w].
 * Right-hand sides are stored [N][nrhs] row-major.
 *
 * The matrix is symmetric and diagonally dominant with positive diagonal,
 * so Gaussian elimination needs no row exchanges; a pivot that is not
 * finite and positive is reported (return value k+1 for pivot k).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

long band_lu(long N, long w, double* ab, double* min_pivot)
{
    const long ld = 2 * w + 1;
    double minp = INFINITY;
    for (long k = 0; k < N; ++k) {
        const double* rk = ab + k * ld;
        const double p = rk[w];
        if (!(p > 0.0) || !isfinite(p)) return k + 1;
        if (p < minp) minp = p;
        const long last = (k + w < N - 1) ? k + w : N - 1;
        for (long r = k + 1; r <= last; ++r) {
            double* rr = ab + r * ld;
            const double l = rr[k - r + w] / p;
            rr[k - r + w] = l;                 /* multiplier, stored in L */
            if (l == 0.0) continue;            /* outside row r's profile */
            for (long c = k + 1; c <= last; ++c)
                rr[c - r + w] -= l * rk[c - k + w];
        }
    }
    if (min_pivot) *min_pivot = minp;
    return 0;
}

void band_solve(long N, long w, const double* ab, long nrhs, double* x)
{
    const long ld = 2 * w + 1;
    /* L y = b, L unit lower */
    for (long r = 0; r < N; ++r) {
        double* xr = x + r * nrhs;
        const long first = (r - w > 0) ? r - w : 0;
        for (long k = first; k < r; ++k) {
            const double l = ab[r * ld + k - r + w];
            if (l == 0.0) continue;
            const double* xk = x + k * nrhs;
            for (long b = 0; b < nrhs; ++b) xr[b] -= l * xk[b];
        }
    }
    /* U x = y */
    for (long r = N - 1; r >= 0; --r) {
        double* xr = x + r * nrhs;
        const long last = (r + w < N - 1) ? r + w : N - 1;
        for (long c = r + 1; c <= last; ++c) {
            const double u = ab[r * ld + c - r + w];
            if (u == 0.0) continue;
            const double* xc = x + c * nrhs;
            for (long b = 0; b < nrhs; ++b) xr[b] -= u * xc[b];
        }
        const double d = ab[r * ld + w];
        for (long b = 0; b < nrhs; ++b) xr[b] /= d;
    }
}

/*
 * out[node][b] = (current injected into node by the sources)
 *              - (current leaving node through its resistors), i.e. the
 * KCL imbalance of node voltages x, accumulated in long double and rounded
 * to double at the end.  V is [nrhs][m]; resistor endpoint b < 0 = ground.
 */
void netlist_residual_ld(long N, long nres, const int64_t* ra, const int64_t* rb,
                         const double* rg, long nsrc, const int64_t* snode,
                         const int64_t* srow, const double* sg, long m,
                         const double* V, long nrhs, const double* x,
                         long double* acc, double* out)
{
    for (long i = 0; i < N * nrhs; ++i) acc[i] = 0.0L;
    for (long e = 0; e < nres; ++e) {
        const long a = (long)ra[e], bn = (long)rb[e];
        const long double g = (long double)rg[e];
        const double* xa = x + a * nrhs;
        long double* aa = acc + a * nrhs;
        if (bn >= 0) {
            const double* xb = x + bn * nrhs;
            long double* ab_ = acc + bn * nrhs;
            for (long b = 0; b < nrhs; ++b) {
                const long double cur = g * ((long double)xa[b] - (long double)xb[b]);
                aa[b] -= cur;
                ab_[b] += cur;
            }
        } else {
            for (long b = 0; b < nrhs; ++b) aa[b] -= g * (long double)xa[b];
        }
    }
    for (long s = 0; s < nsrc; ++s) {
        const long a = (long)snode[s];
        const long i = (long)srow[s];
        const long double g = (long double)sg[s];
        const double* xa = x + a * nrhs;
        long double* aa = acc + a * nrhs;
        for (long b = 0; b < nrhs; ++b)
            aa[b] += g * ((long double)V[b * m + i] - (long double)xa[b]);
    }
    (void)m;
    for (long i = 0; i < N * nrhs; ++i) out[i] = (double)acc[i];
}

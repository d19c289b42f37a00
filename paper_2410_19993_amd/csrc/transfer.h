// Float64 matrix-core product I = V T used by the transfer-matrix shortcut.
#pragma once

#include <hip/hip_runtime.h>

// I[B][n] = V[B][m] T[m][n], all row-major float64 device arrays that do not
// overlap I.  Any B, m >= 1 and 1 <= n; queued on s.
hipError_t xbk_launch_transfer_apply(int B, int m, int n, const double* V, const double* T, double* I,
                                     hipStream_t s);

// One product of fragment-tiled (FRG) n_p x n_p float64 blocks: out = alpha A B^T + C
// (C may be null or equal to out).  Up to two independent products per launch.
struct XbkFrgJob {
    const double* A;
    const double* B;
    const double* C;
    double* out;
};
hipError_t xbk_launch_frg_products(const XbkFrgJob* jobs, int njobs, int n_p, double alpha, hipStream_t s);

// T[i][j] = g_sense sum_{k < n} W_i[j][k] c_i[k] for i < m, j < n: W [m] FRG blocks of
// n_p x n_p, c [m][n_p], T [m][n] row-major.
hipError_t xbk_launch_transfer_rows(int m, int n, int n_p, const double* W, const double* c, double g_sense,
                                    double* T, hipStream_t s);

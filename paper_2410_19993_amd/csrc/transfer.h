// Float64 matrix-core product I = V T used by the transfer-matrix shortcut.
#pragma once

#include <hip/hip_runtime.h>

// I[B][n] = V[B][m] T[m][n], all row-major float64 device arrays that do not
// overlap I.  Any B, m >= 1 and 1 <= n; queued on s.
hipError_t xbk_launch_transfer_apply(int B, int m, int n, const double* V, const double* T, double* I,
                                     hipStream_t s);

// Batched small crossbars: output currents, one workgroup per crossbar.
#pragma once

#include <hip/hip_runtime.h>

// T crossbars of m x n (n <= 64), B <= 256 input vectors each: G [T][m][n],
// V [T][B][m], I [T][B][n], float64 device arrays, I not overlapping G or V.
// block: padded block size (16, 32 or 64, >= n; 0 picks the smallest); split: 1..4
// workgroups per crossbar, each over a contiguous share of its input vectors; unit:
// input vector b is the unit vector e_b (V is not read, B <= m).
hipError_t xbk_launch_tile_currents(int T, int m, int n, int B, double g_wl, double g_bl, double g_src,
                                    double g_sense, const double* G, const double* V, double* I, hipStream_t s,
                                    int block = 0, int split = 1, bool unit = false);

// chasm_obs.hpp -- item rows of the observables of Sec. 5 (the reduced Wigner functions
// W_j and the spatial marginal P), in one canonical summation order.
//
// One FP64 row per item (b, k) of a field with n0 x n1 x n2 x-nodes:
//   q[c]        c = x2 * n0 + x1 < n0 n1: the sum of f over x3 = 0 .. n2-1, in
//               ascending x3;
//   G[g][x3]    g < ceil(n0 n1 / 64): the sum of f at x3 over the 64 columns
//               c = 64 g .. 64 g + 63 (columns beyond the plane count as 0), formed by
//               obs_wave_sum with column 64 g + l in lane l, taken from lane 0.
// W1, W2 and P follow from q, W3 from G (chasm_marginals.hip sums the rows of all items
// in a fixed order).  Every kernel that writes rows -- the separate pass of
// chasm_advect_marginals and the fused epilogues of the x3 sweep that ends an observed
// step -- forms them in exactly this order from the same stored values, so the
// observables are bitwise equal whichever kernel wrote the rows.
#pragma once
#include <hip/hip_runtime.h>

namespace chasm {

__host__ __device__ inline long long obs_groups(int n0, int n1) { return ((long long)n0 * n1 + 63) / 64; }

__host__ __device__ inline long long obs_row(int n0, int n1, int n2)
{
    return (long long)n0 * n1 + obs_groups(n0, n1) * n2;
}

// Butterfly over the 64 lanes of a wave (offsets 32, 16, ..., 1); lane 0's result is
// the canonical sum of a column group.
__device__ __forceinline__ double obs_wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

}  // namespace chasm

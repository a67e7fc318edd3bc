// chasm_marginals.hip -- the visualisation observables of Sec. 5: the reduced Wigner
// functions W_j(x_j, k_j) = integral of f over the other four variables, and the
// spatial marginal P(x1, x2) = integral of f over x3 and k, on the handle's field.
//
// Two passes, FP64, deterministic:
//   k_marg_item   one block per item (the x-cube of one (b, k)): the item's row of
//                 chasm_obs.hpp (column sums q over x3, plane sums G of 64-column
//                 groups), read once from HBM; each wave takes one 64-column group at
//                 a time, so every load of a wave is a contiguous run of x1;
//   k_marg_sum    one thread per output value, summing the item rows in a fixed order
//                 and scaling by the cell volume of the integrated variables.
// The x3 sweep that ends an observed step (CHASM_FLAG_OBSERVE) writes the same rows in
// its epilogue; k_marg_sum then completes the observables without reading the field.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/chasm_advect.h"
#include "chasm_obs.hpp"

namespace chasm {

template <typename T>
__global__ __launch_bounds__(256) void k_marg_item(const T* __restrict__ f, int n0, int n1, int n2,
                                                   double* __restrict__ part)
{
    const int plane = n0 * n1;
    const long long ngr = obs_groups(n0, n1);
    const long long item = blockIdx.x;
    const T* src = f + item * (long long)plane * n2;
    double* q = part + item * obs_row(n0, n1, n2);
    double* G = q + plane;
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    for (long long g = wv; g < ngr; g += 4) {
        const long long c = 64 * g + ln;
        const bool in = c < plane;
        double acc = 0.0;
        for (int z = 0; z < n2; ++z) {
            const double x = in ? (double)src[(long long)z * plane + c] : 0.0;
            acc += x;
            const double gs = obs_wave_sum(x);
            if (ln == 0) G[g * n2 + z] = gs;
        }
        if (in) q[c] = acc;
    }
}

struct MargArgs {
    int nx[3], nk[3], nbatch;
    double s[4];                 // cell volumes of the integrated variables: W1, W2, W3, P
};

// out layout per batch member b: W1[k1][x1] | W2[k2][x2] | W3[k3][x3] | P[x2][x1].
// Per item: W1 takes a[x1] = sum over x2 of q (ascending x2), W2 b[x2] = sum over x1 of
// q (ascending x1), W3 c[x3] = sum over the groups of G (ascending), P the q itself;
// the items are summed k3 outermost, then k2, then k1.
__global__ __launch_bounds__(256) void k_marg_sum(const double* __restrict__ part, MargArgs a,
                                                  double* __restrict__ out)
{
    const int N0 = a.nx[0], N1 = a.nx[1], N2 = a.nx[2], n1 = a.nk[0], n2 = a.nk[1], n3 = a.nk[2];
    const long long ROW = obs_row(N0, N1, N2);
    const long long NG = obs_groups(N0, N1);
    const long long plane = (long long)N0 * N1;
    const long long per_b = (long long)N0 * n1 + (long long)N1 * n2 + (long long)N2 * n3 + plane;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= per_b * a.nbatch) return;
    const int b = (int)(gid / per_b);
    long long r = gid % per_b;
    const double* base = part + (long long)b * n1 * n2 * n3 * ROW;
    auto item = [&](int k1, int k2, int k3) { return base + (((long long)k3 * n2 + k2) * n1 + k1) * ROW; };
    double s = 0.0, scale;
    if (r < (long long)N0 * n1) {
        const int k1 = (int)(r / N0), x = (int)(r % N0);
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k2 = 0; k2 < n2; ++k2) {
                const double* q = item(k1, k2, k3);
                double t = 0.0;
                for (int y = 0; y < N1; ++y) t += q[(long long)y * N0 + x];
                s += t;
            }
        scale = a.s[0];
    } else if ((r -= (long long)N0 * n1) < (long long)N1 * n2) {
        const int k2 = (int)(r / N1), y = (int)(r % N1);
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k1 = 0; k1 < n1; ++k1) {
                const double* q = item(k1, k2, k3) + (long long)y * N0;
                double t = 0.0;
                for (int x = 0; x < N0; ++x) t += q[x];
                s += t;
            }
        scale = a.s[1];
    } else if ((r -= (long long)N1 * n2) < (long long)N2 * n3) {
        const int k3 = (int)(r / N2), z = (int)(r % N2);
        for (int k2 = 0; k2 < n2; ++k2)
            for (int k1 = 0; k1 < n1; ++k1) {
                const double* G = item(k1, k2, k3) + plane;
                double t = 0.0;
                for (long long g = 0; g < NG; ++g) t += G[g * N2 + z];
                s += t;
            }
        scale = a.s[2];
    } else {
        r -= (long long)N2 * n3;                         // (x2, x1) = r
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k2 = 0; k2 < n2; ++k2)
                for (int k1 = 0; k1 < n1; ++k1) s += item(k1, k2, k3)[r];
        scale = a.s[3];
    }
    out[gid] = s * scale;
}

// Rows of FP64 item partials the marginals need per item (chasm_obs.hpp).
long long marginal_row(const int nx[3]) { return obs_row(nx[0], nx[1], nx[2]); }

// Both passes on stream st: part holds nitems * marginal_row(nx) doubles, out
// nbatch * (nx1 nk1 + nx2 nk2 + nx3 nk3 + nx1 nx2) doubles.  f nullptr: the item rows
// are already in part (written by an observing x3 sweep); only the sums run.
hipError_t launch_marginals(int dtype, const int nx[3], const int nk[3], int nbatch, const double hx[3],
                            const double hk[3], const void* f, double* part, double* out, hipStream_t st)
{
    const long long nitems = (long long)nk[0] * nk[1] * nk[2] * nbatch;
    if (f) {
        if (dtype == CHASM_F64)
            hipLaunchKernelGGL((k_marg_item<double>), dim3((unsigned)nitems), dim3(256), 0, st,
                               static_cast<const double*>(f), nx[0], nx[1], nx[2], part);
        else
            hipLaunchKernelGGL((k_marg_item<float>), dim3((unsigned)nitems), dim3(256), 0, st,
                               static_cast<const float*>(f), nx[0], nx[1], nx[2], part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    MargArgs a{};
    a.nbatch = nbatch;
    for (int d = 0; d < 3; ++d) {
        a.nx[d] = nx[d];
        a.nk[d] = nk[d];
    }
    const double v[3] = {hx[0] * hk[0], hx[1] * hk[1], hx[2] * hk[2]};
    a.s[0] = v[1] * v[2];
    a.s[1] = v[0] * v[2];
    a.s[2] = v[0] * v[1];
    a.s[3] = hx[2] * hk[0] * hk[1] * hk[2];
    const long long total = ((long long)nx[0] * nk[0] + (long long)nx[1] * nk[1] + (long long)nx[2] * nk[2] +
                             (long long)nx[0] * nx[1]) * nbatch;
    hipLaunchKernelGGL(k_marg_sum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, a, out);
    return hipGetLastError();
}

}  // namespace chasm

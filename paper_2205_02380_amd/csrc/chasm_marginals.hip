// chasm_marginals.hip -- the visualisation observables of Sec. 5: the reduced Wigner
// functions W_j(x_j, k_j) = integral of f over the other four variables, and the
// spatial marginal P(x1, x2) = integral of f over x3 and k, on the handle's field.
//
// Two passes, FP64, deterministic:
//   k_marg_item   one block per item (the x-cube of one (b, k)): the item's line sums
//                 a[x1] = sum_{x2,x3} f, b[x2] = sum_{x1,x3} f, c[x3] = sum_{x1,x2} f and
//                 its column sums q[x2][x1] = sum_{x3} f, read once from HBM (threads own
//                 (x1, x2) columns, so every load of a wave is a contiguous run of x1);
//   k_marg_sum    one thread per output value, summing the item rows in a fixed order
//                 and scaling by the cell volume of the integrated variables.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/chasm_advect.h"

namespace chasm {

template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_marg_item(const T* __restrict__ f, double* __restrict__ part)
{
    constexpr int ROW = 3 * N + N * N;
    constexpr int NW = NT / 64;
    __shared__ double Q[N * N];
    __shared__ double PW[NW][N];
    const long long item = blockIdx.x;
    const T* src = f + item * (long long)(N * N * N);
    double pl[N];
#pragma unroll
    for (int z = 0; z < N; ++z) pl[z] = 0.0;
    for (int c = threadIdx.x; c < N * N; c += NT) {
        double q = 0.0;
#pragma unroll
        for (int z = 0; z < N; ++z) {
            const double v = (double)src[(long long)z * N * N + c];
            q += v;
            pl[z] += v;
        }
        Q[c] = q;
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
    for (int z = 0; z < N; ++z) {
        double x = pl[z];
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
        if (ln == 0) PW[wv][z] = x;
    }
    __syncthreads();
    double* out = part + item * (long long)ROW;
    if (threadIdx.x < N) {
        const int t = threadIdx.x;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int y = 0; y < N; ++y) a += Q[y * N + t];      // a[x1 = t]
        for (int x = 0; x < N; ++x) b += Q[t * N + x];      // b[x2 = t]
        for (int w = 0; w < NW; ++w) c += PW[w][t];         // c[x3 = t]
        out[t] = a;
        out[N + t] = b;
        out[2 * N + t] = c;
    }
    for (int c = threadIdx.x; c < N * N; c += NT) out[3 * N + c] = Q[c];
}

// Runtime-shape form of k_marg_item for any (n0, n1, n2): one block per item, the
// same row layout (a[x1] | b[x2] | c[x3] | q[x2][x1]), fixed summation orders.
// Columns q first (threads own (x1, x2) columns), then the x3-plane sums c (every
// wave sums its columns of a plane, the waves' sums added in order), then a and b
// from the stored q (the block's own global writes, visible after the barrier).
template <typename T>
__global__ __launch_bounds__(256) void k_marg_item_rt(const T* __restrict__ f, int n0, int n1, int n2,
                                                      double* __restrict__ part)
{
    __shared__ double PW[4];
    const long long plane = (long long)n0 * n1;
    const long long item = blockIdx.x;
    const long long ROW = (long long)n0 + n1 + n2 + plane;
    const T* src = f + item * plane * n2;
    double* out = part + item * ROW;
    double* q = out + n0 + n1 + n2;
    for (long long c = threadIdx.x; c < plane; c += 256) {
        double acc = 0.0;
        for (int z = 0; z < n2; ++z) acc += (double)src[z * plane + c];
        q[c] = acc;
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    for (int z = 0; z < n2; ++z) {
        double x = 0.0;
        for (long long c = threadIdx.x; c < plane; c += 256) x += (double)src[z * plane + c];
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
        if (ln == 0) PW[wv] = x;
        __syncthreads();
        if (threadIdx.x == 0) out[n0 + n1 + z] = PW[0] + PW[1] + PW[2] + PW[3];
        __syncthreads();
    }
    for (int t = threadIdx.x; t < n0; t += 256) {
        double a = 0.0;
        for (int y = 0; y < n1; ++y) a += q[(long long)y * n0 + t];
        out[t] = a;
    }
    for (int t = threadIdx.x; t < n1; t += 256) {
        double b = 0.0;
        for (int x = 0; x < n0; ++x) b += q[(long long)t * n0 + x];
        out[n0 + t] = b;
    }
}

struct MargArgs {
    int nx[3], nk[3], nbatch;
    double s[4];                 // cell volumes of the integrated variables: W1, W2, W3, P
};

// out layout per batch member b: W1[k1][x1] | W2[k2][x2] | W3[k3][x3] | P[x2][x1]
__global__ __launch_bounds__(256) void k_marg_sum(const double* __restrict__ part, MargArgs a,
                                                  double* __restrict__ out)
{
    const int N0 = a.nx[0], N1 = a.nx[1], N2 = a.nx[2], n1 = a.nk[0], n2 = a.nk[1], n3 = a.nk[2];
    const long long ROW = (long long)N0 + N1 + N2 + (long long)N0 * N1;
    const long long per_b = (long long)N0 * n1 + (long long)N1 * n2 + (long long)N2 * n3 + (long long)N0 * N1;
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
            for (int k2 = 0; k2 < n2; ++k2) s += item(k1, k2, k3)[x];
        scale = a.s[0];
    } else if ((r -= (long long)N0 * n1) < (long long)N1 * n2) {
        const int k2 = (int)(r / N1), x = (int)(r % N1);
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k1 = 0; k1 < n1; ++k1) s += item(k1, k2, k3)[N0 + x];
        scale = a.s[1];
    } else if ((r -= (long long)N1 * n2) < (long long)N2 * n3) {
        const int k3 = (int)(r / N2), x = (int)(r % N2);
        for (int k2 = 0; k2 < n2; ++k2)
            for (int k1 = 0; k1 < n1; ++k1) s += item(k1, k2, k3)[N0 + N1 + x];
        scale = a.s[2];
    } else {
        r -= (long long)N2 * n3;                         // (x2, x1) = r
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k2 = 0; k2 < n2; ++k2)
                for (int k1 = 0; k1 < n1; ++k1) s += item(k1, k2, k3)[N0 + N1 + N2 + r];
        scale = a.s[3];
    }
    out[gid] = s * scale;
}

template <typename T, int N>
static hipError_t launch_item(const void* f, long long nitems, double* part, hipStream_t st)
{
    constexpr int NT = 256;
    hipLaunchKernelGGL((k_marg_item<T, N, NT>), dim3((unsigned)nitems), dim3(NT), 0, st, static_cast<const T*>(f), part);
    return hipGetLastError();
}

// Item rows: the compiled form for the cubic grids it is built for, else the runtime one.
template <typename T>
static hipError_t launch_item_n(const int nx[3], const void* f, long long nitems, double* part, hipStream_t st)
{
    if (nx[0] == nx[1] && nx[0] == nx[2]) {
        switch (nx[0]) {
            case 8: return launch_item<T, 8>(f, nitems, part, st);
            case 16: return launch_item<T, 16>(f, nitems, part, st);
            case 24: return launch_item<T, 24>(f, nitems, part, st);
            case 32: return launch_item<T, 32>(f, nitems, part, st);
            case 48: return launch_item<T, 48>(f, nitems, part, st);
            case 64: return launch_item<T, 64>(f, nitems, part, st);
            default: break;
        }
    }
    hipLaunchKernelGGL((k_marg_item_rt<T>), dim3((unsigned)nitems), dim3(256), 0, st, static_cast<const T*>(f), nx[0],
                       nx[1], nx[2], part);
    return hipGetLastError();
}

// Rows of FP64 item partials the marginals need (n0 + n1 + n2 + n0 n1 per item).
long long marginal_row(const int nx[3]) { return (long long)nx[0] + nx[1] + nx[2] + (long long)nx[0] * nx[1]; }

// Both passes on stream st: part holds nitems * marginal_row(nx) doubles, out
// nbatch * (nx1 nk1 + nx2 nk2 + nx3 nk3 + nx1 nx2) doubles.
hipError_t launch_marginals(int dtype, const int nx[3], const int nk[3], int nbatch, const double hx[3],
                            const double hk[3], const void* f, double* part, double* out, hipStream_t st)
{
    const long long nitems = (long long)nk[0] * nk[1] * nk[2] * nbatch;
    hipError_t e = dtype == CHASM_F64 ? launch_item_n<double>(nx, f, nitems, part, st)
                                      : launch_item_n<float>(nx, f, nitems, part, st);
    if (e != hipSuccess) return e;
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

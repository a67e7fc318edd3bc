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

struct MargArgs {
    int N, nk[3], nbatch;
    double s[4];                 // cell volumes of the integrated variables: W1, W2, W3, P
};

// out layout per batch member b: W1[k1][x1] | W2[k2][x2] | W3[k3][x3] | P[x2][x1]
__global__ __launch_bounds__(256) void k_marg_sum(const double* __restrict__ part, MargArgs a,
                                                  double* __restrict__ out)
{
    const int N = a.N, n1 = a.nk[0], n2 = a.nk[1], n3 = a.nk[2];
    const long long ROW = 3LL * N + (long long)N * N;
    const long long per_b = (long long)N * (n1 + n2 + n3) + (long long)N * N;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= per_b * a.nbatch) return;
    const int b = (int)(gid / per_b);
    long long r = gid % per_b;
    const double* base = part + (long long)b * n1 * n2 * n3 * ROW;
    auto item = [&](int k1, int k2, int k3) { return base + (((long long)k3 * n2 + k2) * n1 + k1) * ROW; };
    double s = 0.0, scale;
    if (r < (long long)N * n1) {
        const int k1 = (int)(r / N), x = (int)(r % N);
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k2 = 0; k2 < n2; ++k2) s += item(k1, k2, k3)[x];
        scale = a.s[0];
    } else if ((r -= (long long)N * n1) < (long long)N * n2) {
        const int k2 = (int)(r / N), x = (int)(r % N);
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k1 = 0; k1 < n1; ++k1) s += item(k1, k2, k3)[N + x];
        scale = a.s[1];
    } else if ((r -= (long long)N * n2) < (long long)N * n3) {
        const int k3 = (int)(r / N), x = (int)(r % N);
        for (int k2 = 0; k2 < n2; ++k2)
            for (int k1 = 0; k1 < n1; ++k1) s += item(k1, k2, k3)[2 * N + x];
        scale = a.s[2];
    } else {
        r -= (long long)N * n3;                          // (x2, x1) = r
        for (int k3 = 0; k3 < n3; ++k3)
            for (int k2 = 0; k2 < n2; ++k2)
                for (int k1 = 0; k1 < n1; ++k1) s += item(k1, k2, k3)[3 * N + r];
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

template <typename T>
static hipError_t launch_item_n(int N, const void* f, long long nitems, double* part, hipStream_t st)
{
    switch (N) {
        case 8: return launch_item<T, 8>(f, nitems, part, st);
        case 16: return launch_item<T, 16>(f, nitems, part, st);
        case 24: return launch_item<T, 24>(f, nitems, part, st);
        case 32: return launch_item<T, 32>(f, nitems, part, st);
        case 48: return launch_item<T, 48>(f, nitems, part, st);
        case 64: return launch_item<T, 64>(f, nitems, part, st);
        default: return hipErrorInvalidValue;
    }
}

// Rows of FP64 item partials the marginals need (3N + N^2 per item).
long long marginal_row(int N) { return 3LL * N + (long long)N * N; }

// Both passes on stream st: part holds nitems * marginal_row(N) doubles, out
// nbatch * (N (nk1 + nk2 + nk3) + N^2) doubles.
hipError_t launch_marginals(int dtype, int N, const int nk[3], int nbatch, const double hx[3], const double hk[3],
                            const void* f, double* part, double* out, hipStream_t st)
{
    const long long nitems = (long long)nk[0] * nk[1] * nk[2] * nbatch;
    hipError_t e = dtype == CHASM_F64 ? launch_item_n<double>(N, f, nitems, part, st)
                                      : launch_item_n<float>(N, f, nitems, part, st);
    if (e != hipSuccess) return e;
    MargArgs a{};
    a.N = N;
    a.nbatch = nbatch;
    for (int d = 0; d < 3; ++d) a.nk[d] = nk[d];
    const double v[3] = {hx[0] * hk[0], hx[1] * hk[1], hx[2] * hk[2]};
    a.s[0] = v[1] * v[2];
    a.s[1] = v[0] * v[2];
    a.s[2] = v[0] * v[1];
    a.s[3] = hx[2] * hk[0] * hk[1] * hk[2];
    const long long total = ((long long)N * (nk[0] + nk[1] + nk[2]) + (long long)N * N) * nbatch;
    hipLaunchKernelGGL(k_marg_sum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, a, out);
    return hipGetLastError();
}

}  // namespace chasm

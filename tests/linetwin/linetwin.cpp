// Host twin of the kernel line algebra, for CPU tests only.
//
// Compiles the library's own line routine (chasm_line.hpp: compile-time PMBC rows and
// patch factors, register line solve, shifted store) and its FP64 table builder
// (chasm_tables.cpp: per-k shift weights, host stencil rows) for the host, in FP64 and
// FP32, so the tests can compare the HIP path's arithmetic with the oracle without a
// GPU.  Never linked into the product.
#include <cstring>
#include <string>

#include "../../paper_2205_02380_amd/csrc/chasm_line.hpp"
#include "../../paper_2205_02380_amd/csrc/chasm_tables.hpp"

using namespace chasm;

template <typename T, int N, int M, int G, int CL>
static int run(double h, int nk, double klo, double hk, double dt, int ik, const double* phi, double* out)
{
    AxisTables t;
    std::string err;
    if (!build_axis_tables(N, M, G, G, h, CL, nk, klo, hk, dt, t, err)) return -1;
    AxisCoef<T> k;
    k.w0 = (T)t.w[4 * ik + 0];
    k.w1 = (T)t.w[4 * ik + 1];
    k.w2 = (T)t.w[4 * ik + 2];
    k.w3 = (T)t.w[4 * ik + 3];
    T v[N];
    for (int i = 0; i < N; ++i) v[i] = (T)phi[i];
    T res[N];
    const int sigma = t.shift[ik];
    dispatch_sigma(sigma, [&](auto sc) {
        advect_line<T, N, M, G, CL, decltype(sc)::value>(v, k, sigma, [&](int j, T x) { res[j] = x; });
    });
    for (int i = 0; i < N; ++i) out[i] = (double)res[i];
    return 0;
}

template <int N, int M, int G, int CL>
static int rows(double* out)
{
    constexpr Stencil<N, M, G, CL> st{};
    constexpr int W = 2 * G + 1;
    for (int q = 0; q <= Shape<N, M>::P; ++q)
        for (int t = 0; t < W; ++t) out[q * W + t] = st.c[q][t];
    return 0;
}

#define SHAPES(X)                                                                                  \
    X(8, 2, 1, 0) X(8, 4, 3, 0) X(8, 4, 3, 1) X(8, 8, 7, 0) X(8, 8, 7, 1) X(16, 8, 4, 0) X(16, 8, 4, 1)    \
    X(16, 8, 15, 0) X(16, 5, 6, 0) X(16, 5, 6, 1) X(24, 8, 6, 0) X(24, 8, 6, 1) X(32, 8, 6, 0)            \
    X(32, 8, 6, 1) X(48, 16, 8, 0) X(48, 16, 8, 1) X(64, 16, 8, 0) X(64, 16, 8, 1) X(61, 15, 8, 0)        \
    X(61, 15, 8, 1) X(8, 4, 3, 2) X(16, 8, 4, 2) X(16, 8, 15, 2) X(32, 8, 6, 2) X(61, 15, 8, 2)

// One sweep of one line with shift alpha = k dt / h for the single k = klo.
extern "C" int twin_line(int fp64, int N, int M, int G, int CL, double h, double klo, double dt,
                         const double* phi, double* out)
{
#define X(NN, MM, GG, CC)                                                                         \
    if (N == NN && M == MM && G == GG && CL == CC)                                                 \
        return fp64 ? run<double, NN, MM, GG, CC>(h, 1, klo, 1.0, dt, 0, phi, out)                 \
                    : run<float, NN, MM, GG, CC>(h, 1, klo, 1.0, dt, 0, phi, out);
    SHAPES(X)
#undef X
    return -2;
}

// The compile-time interface rows (times h) of a shape: (P+1) x (2G+1).
extern "C" int twin_rows(int N, int M, int G, int CL, double* out)
{
#define X(NN, MM, GG, CC) \
    if (N == NN && M == MM && G == GG && CL == CC) return rows<NN, MM, GG, CC>(out);
    SHAPES(X)
#undef X
    return -2;
}

// The host FP64 table rows of a shape (the same rows, from chasm_tables.cpp).
extern "C" int twin_host_rows(int N, int M, int G, int CL, double h, double* out)
{
    AxisTables t;
    std::string err;
    if (!build_axis_tables(N, M, G, G, h, CL, 1, 0.0, 1.0, 0.0, t, err)) return -1;
    std::memcpy(out, t.stencil.data(), t.stencil.size() * sizeof(double));
    return 0;
}

// Host twin of the kernel line algebra, for CPU tests only.
//
// Compiles the library's own line routine (chasm_line.hpp) and table builder
// (chasm_tables.cpp) for the host in FP64 and FP32, so the tests can compare the
// HIP path's arithmetic with the oracle without a GPU.  Never linked into the product.
#include <cstring>
#include <string>

#include "../../paper_2205_02380_amd/csrc/chasm_line.hpp"
#include "../../paper_2205_02380_amd/csrc/chasm_tables.hpp"

using namespace chasm;

template <typename T, int N, int M, int G>
static int run(int g, double h, int closure, int nk, double klo, double hk, double dt, int ik, const double* phi,
               double* out)
{
    AxisTables t;
    std::string err;
    if (!build_axis_tables(N, M, g, G, h, closure, nk, klo, hk, dt, t, err)) return -1;
    T st[(Shape<N, M>::P + 1) * (2 * G + 1)], fac[6 * (M + 1)];
    for (size_t i = 0; i < t.stencil.size(); ++i) st[i] = (T)t.stencil[i];
    for (size_t i = 0; i < t.fac.size(); ++i) fac[i] = (T)t.fac[i];
    AxisCoef<T> k;
    k.stencil = st;
    k.fac = fac;
    k.h3 = (T)(h / 3.0);
    k.twoh = (T)(2.0 * h);
    k.w0 = (T)t.w[4 * ik + 0];
    k.w1 = (T)t.w[4 * ik + 1];
    k.w2 = (T)t.w[4 * ik + 2];
    k.w3 = (T)t.w[4 * ik + 3];
    k.ghost = (T)(closure == 1 ? 1 : 0);
    T v[N], cv[N + 7];
    for (int i = 0; i < N; ++i) v[i] = (T)phi[i];
    line_cells<T, N, M, G>(v, cv, k);
    T res[N];
    store_shifted<T, N>(cv, t.shift[ik], [&](int j, T x) { res[j] = x; });
    for (int i = 0; i < N; ++i) out[i] = (double)res[i];
    return 0;
}

#define SHAPES(X) X(8, 2, 7) X(8, 4, 7) X(16, 8, 8) X(16, 8, 15) X(16, 5, 8) X(24, 8, 8) X(32, 8, 8) X(48, 16, 8) X(64, 16, 8) X(61, 15, 8)

extern "C" int twin_line(int fp64, int N, int M, int G, int g, double h, int closure, int nk, double klo, double hk,
                         double dt, int ik, const double* phi, double* out)
{
#define X(NN, MM, GG)                                                                               \
    if (N == NN && M == MM && G == GG)                                                             \
        return fp64 ? run<double, NN, MM, GG>(g, h, closure, nk, klo, hk, dt, ik, phi, out)         \
                    : run<float, NN, MM, GG>(g, h, closure, nk, klo, hk, dt, ik, phi, out);
    SHAPES(X)
#undef X
    return -2;
}

// chasm_line.hpp -- one patched cubic-spline shift of one line, held in registers.
//
// Method: Xiong, Zhang, Shao, "A characteristic-spectral-mixed scheme for
// six-dimensional Wigner-Coulomb dynamics" (arXiv:2205.02380), Sec. 3.1.
//
// A line of N nodes is split into P patches of M cells that share end nodes
// (eq. 3.1; P = ceil((N-1)/M), the last patch has MLAST <= M cells).  For one line:
//   1. interface slopes (times h) d_q = sum_j c_j(I_q) h v_j at the P+1 interfaces
//      I_q = q*M (q < P) and I_P = N-1: the PMBC rows of eqs. 3.4-3.5 (rows of the
//      natural-BC inverse, truncated to |j - I_q| <= G, G the ghost width).  The rows
//      times h depend only on (N, M, G, closure), so they are compile-time FP64
//      constants rounded once to T;
//   2. per patch, the (m+3)-unknown Hermite system of Sec. 3.1.2 step (5).  Its two
//      slope rows (eq. 2.13) eliminate eta_{-1} and eta_{m+1}, which leaves the
//      diagonally dominant tridiagonal system
//        (2/3 1/3; 1/6 2/3 1/6; ...; 1/3 2/3) eta_{0..m}
//          = (v_0 + (h/3) d_L, v_1, ..., v_{m-1}, v_m - (h/3) d_R),
//      (h d appears only as the product computed in step 1),
//      solved by the sweeping (Thomas) method; its factors depend only on the patch
//      length, so they are compile-time FP64 constants rounded once to T;
//      then eta_{-1} = eta_1 - 2h d_L and eta_{m+1} = eta_{m-1} + 2h d_R;
//   3. cell values: for each cell c (departure points in [x_c, x_{c+1})), the owning
//      patch evaluates w0 eta_{c-1} + w1 eta_c + w2 eta_{c+1} + w3 eta_{c+2}
//      (eqs. 3.7-3.10 with the departure fraction beta: w_r = b_{4-r}(1 - beta)).
//      Cells -4..-1 and N-1..N+2 lie beyond the line ends and use the outer ghost
//      coefficient (0 for the paper's closure, Sec. 3.1.3; a zero fourth difference
//      for the cubic-exact closure).
// The output node j takes the value of cell j + sigma, sigma = floor(-alpha):
// the upwind patch evaluates it (correction procedure, Sec. 3.1.3).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace chasm {

template <int N, int M>
struct Shape {
    static_assert(N >= 2 && M >= 1, "bad line shape");
    static constexpr int P = (N - 1 + M - 1) / M;            // patches
    static constexpr int MLAST = N - 1 - (P - 1) * M;        // cells of the last patch
    __host__ __device__ static constexpr int iface(int q) { return q < P ? q * M : N - 1; }
    __host__ __device__ static constexpr int start(int l) { return l * M; }
    __host__ __device__ static constexpr int cells(int l) { return l == P - 1 ? MLAST : M; }
};

// Compile-time loop: f(std::integral_constant<int, I>{}) for I = B .. E-1.
template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Thomas factors of the reduced patch system of length m+1 (rows scaled by 1/6):
// row 0 (2/3, 1/3), rows 1..m-1 (1/6, 2/3, 1/6), row m (1/3, 2/3).  Forward sweep
// e_i = (r_i - a_i e_{i-1}) / den_i, back substitution eta_i = e_i - c'_i eta_{i+1};
// inv = 1/den, ainv = a/den, cp = c/den.  Evaluated in FP64 at compile time.
template <int m>
struct PatchLU {
    double inv[m + 1] = {}, ainv[m + 1] = {}, cp[m + 1] = {};
    constexpr PatchLU()
    {
        double prev = 0.0;
        for (int i = 0; i <= m; ++i) {
            const double a = (i == 0) ? 0.0 : (i == m ? 1.0 / 3.0 : 1.0 / 6.0);
            const double c = (i == m) ? 0.0 : (i == 0 ? 1.0 / 3.0 : 1.0 / 6.0);
            const double den = 2.0 / 3.0 - a * prev;
            inv[i] = 1.0 / den;
            ainv[i] = a / den;
            cp[i] = c / den;
            prev = cp[i];
        }
    }
};

// PMBC interface rows times h: c[q][t] multiplies v[I_q - G + t] (zero outside the
// line).  The slopes of the natural cubic spline (eq. 2.14) follow from the reduced
// system: eta_0 = phi_0, eta_{N-1} = phi_{N-1}, eta_{i-1} + 4 eta_i + eta_{i+1} = 6 phi_i
// for 0 < i < N-1, eta_{-1} = 2 eta_0 - eta_1, eta_N = 2 eta_{N-1} - eta_{N-2}, and
// h s'(x_I) = (eta_{I+1} - eta_{I-1}) / 2.  Closure CL = 1 adds the minimum-norm
// correction that makes each truncated row exact for cubics (normal equations on the
// scaled monomials ((j-I)/G)^q, q = 0..3).  CL = 2 takes the rows of the Neumann
// global spline instead (see neumann()).  All in FP64 at compile time.
template <int N, int M, int G, int CL>
struct Stencil {
    static constexpr int P = Shape<N, M>::P;
    static constexpr int W = 2 * G + 1;
    double c[P + 1][W] = {};
    constexpr Stencil()
    {
        if constexpr (CL == 2) {
            neumann();
            return;
        }
        constexpr int n = N - 2;
        double cp[N] = {}, den[N] = {};
        for (int i = 0; i < n; ++i) {
            den[i] = 4.0 - (i > 0 ? cp[i - 1] : 0.0);
            cp[i] = 1.0 / den[i];
        }
        for (int j = 0; j < N; ++j) {
            double eta[N + 2] = {}, y[N] = {};
            const double e0 = j == 0 ? 1.0 : 0.0, eN = j == N - 1 ? 1.0 : 0.0;
            eta[1] = e0;
            eta[N] = eN;
            for (int i = 0; i < n; ++i) {
                double r = (j == i + 1) ? 6.0 : 0.0;
                if (i == 0) r -= e0;
                if (i == n - 1) r -= eN;
                y[i] = (r - (i > 0 ? y[i - 1] : 0.0)) / den[i];
            }
            for (int i = n - 1; i >= 0; --i) {
                if (i < n - 1) y[i] -= cp[i] * y[i + 1];
                eta[i + 2] = y[i];
            }
            eta[0] = 2.0 * eta[1] - eta[2];
            eta[N + 1] = 2.0 * eta[N] - eta[N - 1];
            for (int q = 0; q <= P; ++q) {
                const int I = Shape<N, M>::iface(q);
                const int t = j - I + G;
                if (t >= 0 && t < W) c[q][t] = 0.5 * (eta[I + 2] - eta[I]);
            }
        }
        if (CL == 1) {
            for (int q = 0; q <= P; ++q) {
                const int I = Shape<N, M>::iface(q);
                double A[4][5] = {};                    // [V^T V | e - V^T c]
                A[1][4] = 1.0 / G;
                for (int t = 0; t < W; ++t) {
                    const int j = I - G + t;
                    if (j < 0 || j >= N) continue;
                    const double u = (double)(t - G) / G;
                    const double pw[4] = {1.0, u, u * u, u * u * u};
                    for (int a = 0; a < 4; ++a) {
                        A[a][4] -= pw[a] * c[q][t];
                        for (int b = 0; b < 4; ++b) A[a][b] += pw[a] * pw[b];
                    }
                }
                for (int k = 0; k < 4; ++k)             // Gaussian elimination (SPD, no pivoting)
                    for (int r = k + 1; r < 4; ++r) {
                        const double f = A[r][k] / A[k][k];
                        for (int cc = k; cc < 5; ++cc) A[r][cc] -= f * A[k][cc];
                    }
                double lam[4] = {};
                for (int k = 3; k >= 0; --k) {
                    double acc = A[k][4];
                    for (int cc = k + 1; cc < 4; ++cc) acc -= A[k][cc] * lam[cc];
                    lam[k] = acc / A[k][k];
                }
                for (int t = 0; t < W; ++t) {
                    const int j = I - G + t;
                    if (j < 0 || j >= N) continue;
                    const double u = (double)(t - G) / G;
                    c[q][t] += lam[0] + u * (lam[1] + u * (lam[2] + u * lam[3]));
                }
            }
        }
    }

    // CL = 2: the Neumann condition (eq. 2.13 with zero end slopes) gives eta_{-1} =
    // eta_1 and eta_N = eta_{N-2}; with the interpolation rows the unknowns eta_0..eta_{N-1}
    // solve the tridiagonal system [4 2; 1 4 1; ...; 2 4] eta = 6 phi (Thomas, per unit
    // data vector).  The slopes at both line ends are then exactly 0.
    constexpr void neumann()
    {
        double cp[N] = {}, den[N] = {};
        for (int i = 0; i < N; ++i) {
            const double sub = i == N - 1 ? 2.0 : 1.0, sup = i == 0 ? 2.0 : 1.0;
            den[i] = 4.0 - (i > 0 ? sub * cp[i - 1] : 0.0);
            cp[i] = sup / den[i];
        }
        for (int j = 0; j < N; ++j) {
            double eta[N + 2] = {}, y[N] = {};
            for (int i = 0; i < N; ++i) {
                const double sub = i == N - 1 ? 2.0 : 1.0;
                const double r = (i == j) ? 6.0 : 0.0;
                y[i] = (r - (i > 0 ? sub * y[i - 1] : 0.0)) / den[i];
            }
            for (int i = N - 2; i >= 0; --i) y[i] -= cp[i] * y[i + 1];
            for (int i = 0; i < N; ++i) eta[i + 1] = y[i];
            eta[0] = eta[2];
            eta[N + 1] = eta[N - 1];
            for (int q = 0; q <= P; ++q) {
                const int I = Shape<N, M>::iface(q);
                const int t = j - I + G;
                if (t >= 0 && t < W) c[q][t] = 0.5 * (eta[I + 2] - eta[I]);
            }
        }
    }
};

// Shift weights of one line's k (uniform across a work-group).
template <typename T>
struct AxisCoef {
    T w0, w1, w2, w3;
};

// Cell values are stored at cv[c + CV_OFF] for c in [-4, N+2]: the four cells left of
// the line and the four right of it are the ones the outer ghost coefficients reach.
constexpr int CV_OFF = 4;
template <int N>
struct CellCount { static constexpr int value = N + 7; };

// Cell values of one line, handed out as soon as each patch is solved:
// emit(std::integral_constant<int, c>{}, value) for c in [-4, N+2].  Emitting early
// keeps only one patch's coefficients live at a time.
template <typename T, int N, int M, int G, int CL, typename Emit>
__host__ __device__ __forceinline__ void line_emit(const T (&v)[N], const AxisCoef<T>& k, Emit&& emit)
{
    using S = Shape<N, M>;
    constexpr int P = S::P;
    constexpr int W = 2 * G + 1;
    constexpr Stencil<N, M, G, CL> st{};

    // 1. interface slopes times h
    T d[P + 1];
    static_for<0, P + 1>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int I = S::iface(q);
        T acc = T(0);
        static_for<0, W>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            constexpr int j = I - G + t;
            constexpr T cq = (T)st.c[q][t];
            if constexpr (j >= 0 && j < N && cq != T(0)) acc = fma(cq, v[j], acc);
        });
        d[q] = acc;
    });

    static_for<0, P>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        constexpr int s = S::start(l);
        constexpr int m = S::cells(l);
        constexpr PatchLU<m> lu{};

        // 2. forward sweep of the reduced tridiagonal system
        T e[m + 1];
        e[0] = fma(T(1.0 / 3.0), d[l], v[s]) * (T)lu.inv[0];
        static_for<1, m + 1>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr T inv_i = (T)lu.inv[i], ainv_i = (T)lu.ainv[i];
            T r = v[s + i];
            if constexpr (i == m) r = fma(T(-1.0 / 3.0), d[l + 1], r);
            e[i] = fma(-ainv_i, e[i - 1], r * inv_i);
        });
        // back substitution: eta[u] = eta_{u-1}, u = 0..m+2
        T eta[m + 3];
        eta[m + 1] = e[m];
        static_for<0, m>([&](auto ic) {
            constexpr int i = m - 1 - decltype(ic)::value;
            constexpr T cp_i = (T)lu.cp[i];
            eta[i + 1] = fma(-cp_i, eta[i + 2], e[i]);
        });
        eta[0] = fma(T(-2), d[l], eta[2]);
        eta[m + 2] = fma(T(2), d[l + 1], eta[m]);

        // 3. cell values of this patch's cells c = s .. s+m-1 (local nu = c - s)
        static_for<0, m>([&](auto nc) {
            constexpr int nu = decltype(nc)::value;
            T a = k.w0 * eta[nu];
            a = fma(k.w1, eta[nu + 1], a);
            a = fma(k.w2, eta[nu + 2], a);
            a = fma(k.w3, eta[nu + 3], a);
            emit(std::integral_constant<int, s + nu>{}, a);
        });
        if constexpr (l == 0) {
            // beyond the left end: eta_{-2} is the ghost (0, or a zero fourth
            // difference for the cubic-exact closure), further out zero
            const T gl = CL == 1 ? (4 * eta[0] - 6 * eta[1] + 4 * eta[2] - eta[3]) : T(0);
            emit(std::integral_constant<int, -1>{}, fma(k.w3, eta[2], fma(k.w2, eta[1], fma(k.w1, eta[0], k.w0 * gl))));
            emit(std::integral_constant<int, -2>{}, fma(k.w3, eta[1], fma(k.w2, eta[0], k.w1 * gl)));
            emit(std::integral_constant<int, -3>{}, fma(k.w3, eta[0], k.w2 * gl));
            emit(std::integral_constant<int, -4>{}, k.w3 * gl);
        }
        if constexpr (l == P - 1) {
            // beyond the right end: eta_{m+2} is the ghost
            const T gr = CL == 1 ? (4 * eta[m + 2] - 6 * eta[m + 1] + 4 * eta[m] - eta[m - 1]) : T(0);
            emit(std::integral_constant<int, N - 1>{},
                 fma(k.w3, gr, fma(k.w2, eta[m + 2], fma(k.w1, eta[m + 1], k.w0 * eta[m]))));
            emit(std::integral_constant<int, N>{}, fma(k.w2, gr, fma(k.w1, eta[m + 2], k.w0 * eta[m + 1])));
            emit(std::integral_constant<int, N + 1>{}, fma(k.w1, gr, k.w0 * eta[m + 2]));
            emit(std::integral_constant<int, N + 2>{}, k.w0 * gr);
        }
    });
}

// Cell values of one line.  v[N] in, cv[c + CV_OFF] out for c in [-4, N+2].
template <typename T, int N, int M, int G, int CL>
__host__ __device__ __forceinline__ void line_cells(const T (&v)[N], T (&cv)[N + 7], const AxisCoef<T>& k)
{
    line_emit<T, N, M, G, CL>(v, k, [&](auto cc, T x) { cv[decltype(cc)::value + CV_OFF] = x; });
}

// Write output node j = c - sigma for every cell value; nodes whose departure cell
// lies further out than the ghost cells get 0.  st(j, value) performs the store with
// a compile-time j.  sigma is uniform over a work-group for a whole sweep, so callers
// dispatch once per sweep on SIG: 0 and -1 (|alpha| < 1) store straight from the cell
// values; SIG_ANY handles any other shift through a register barrel shifter (one
// stage per bit of |sigma + CV_OFF|, each a compile-time shift selected by that bit).
constexpr int SIG_ANY = 1;

template <typename T, int N, int SIG, typename Store>
__host__ __device__ __forceinline__ void store_cells(const T (&cv)[N + 7], int sigma, Store st)
{
    constexpr int K = N + 7;
    if constexpr (SIG == 0 || SIG == -1) {
        static_for<0, N>([&](auto jc) { st(decltype(jc)::value, cv[decltype(jc)::value + CV_OFF + SIG]); });
    } else {
        // out[j] = cv[j + u] with u = sigma + CV_OFF (zero outside 0..K-1)
        const int u = sigma + CV_OFF;
        const int mag = u < 0 ? -u : u;
        T a[K];
        static_for<0, K>([&](auto ic) { a[decltype(ic)::value] = (mag < K) ? cv[decltype(ic)::value] : T(0); });
        if (u >= 0) {
            static_for<0, 7>([&](auto bc) {
                constexpr int sh = 1 << decltype(bc)::value;
                if (mag & sh) {
                    static_for<0, K>([&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        if constexpr (i + sh < K) a[i] = a[i + sh]; else a[i] = T(0);
                    });
                }
            });
        } else {
            static_for<0, 7>([&](auto bc) {
                constexpr int sh = 1 << decltype(bc)::value;
                if (mag & sh) {
                    static_for<0, K>([&](auto ic) {
                        constexpr int i = K - 1 - decltype(ic)::value;
                        if constexpr (i - sh >= 0) a[i] = a[i - sh]; else a[i] = T(0);
                    });
                }
            });
        }
        static_for<0, N>([&](auto jc) { st(decltype(jc)::value, a[decltype(jc)::value]); });
    }
}

// Run body(std::integral_constant<int, SIG>) with SIG matching sigma's class.
template <typename Body>
__host__ __device__ __forceinline__ void dispatch_sigma(int sigma, Body&& body)
{
    if (sigma == 0) body(std::integral_constant<int, 0>{});
    else if (sigma == -1) body(std::integral_constant<int, -1>{});
    else body(std::integral_constant<int, SIG_ANY>{});
}

// One line, computed and stored: for SIG 0 / -1 each cell value goes straight to its
// output node j = c - SIG (compile time) as soon as its patch is solved.  For any
// other shift the destination j = c - sigma is a runtime value, uniform across the
// work-group; every in-range destination is stored once and the nodes whose
// departure cell lies beyond the ghost cells get 0.  st(j, x) stores one node.
template <typename T, int N, int M, int G, int CL, int SIG, typename Store>
__host__ __device__ __forceinline__ void advect_line(const T (&v)[N], const AxisCoef<T>& k, int sigma, Store st)
{
    if constexpr (SIG == 0 || SIG == -1) {
        line_emit<T, N, M, G, CL>(v, k, [&](auto cc, T x) {
            constexpr int j = decltype(cc)::value - SIG;
            if constexpr (j >= 0 && j < N) st(j, x);
        });
    } else {
        line_emit<T, N, M, G, CL>(v, k, [&](auto cc, T x) {
            const int j = decltype(cc)::value - sigma;
            if (j >= 0 && j < N) st(j, x);
        });
        for (int j = 0; j < N; ++j) {
            const int c = j + sigma;
            if (c < -CV_OFF || c > N + 2) st(j, T(0));
        }
    }
}

// Convenience form with the dispatch inside (one line; used off the hot loops).
template <typename T, int N, typename Store>
__host__ __device__ __forceinline__ void store_shifted(const T (&cv)[N + 7], int sigma, Store st)
{
    dispatch_sigma(sigma, [&](auto sc) { store_cells<T, N, decltype(sc)::value>(cv, sigma, st); });
}

}  // namespace chasm

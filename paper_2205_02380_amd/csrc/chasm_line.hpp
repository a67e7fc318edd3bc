// chasm_line.hpp -- one patched cubic-spline shift of one line, held in registers.
//
// Method: Xiong, Zhang, Shao, "A characteristic-spectral-mixed scheme for
// six-dimensional Wigner-Coulomb dynamics" (arXiv:2205.02380), Sec. 3.1.
//
// A line of N nodes is split into P patches of M cells that share end nodes
// (eq. 3.1; P = ceil((N-1)/M), the last patch has MLAST <= M cells).  For one line:
//   1. interface slopes d_q = sum_t S[q][t] v[I_q - G + t] at the P+1 interfaces
//      I_q = q*M (q < P) and I_P = N-1: the truncated PMBC rows of eqs. 3.4-3.5,
//      stored densely over the window [I_q - G, I_q + G] (zeros past the actual
//      ghost width g <= G and outside the line);
//   2. per patch, the (m+3)-unknown Hermite system of Sec. 3.1.2 step (5).  Its two
//      slope rows (eq. 2.13) eliminate eta_{-1} and eta_{m+1}, which leaves the
//      diagonally dominant tridiagonal system
//        (2/3 1/3; 1/6 2/3 1/6; ...; 1/3 2/3) eta_{0..m}
//          = (v_0 + (h/3) d_L, v_1, ..., v_{m-1}, v_m - (h/3) d_R),
//      solved by the sweeping (Thomas) method with host-built FP64 factors;
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

// Per-axis coefficients as seen by one line (uniform across a work-group).  Ptr is the
// table pointer type: kernels read through the constant address space so the
// compiler keeps the coefficients in SGPRs (scalar loads); host builds use const T*.
template <typename T, typename Ptr = const T*>
struct AxisCoef {
    Ptr stencil;                     // [(P+1)][2G+1]
    Ptr fac;                         // [2][3][MF]: inv, a*inv, c' for m = M (0), m = MLAST (1)
    T h3;                            // h/3
    T twoh;                          // 2h
    T w0, w1, w2, w3;                // shift weights of this line's k
    T ghost;                         // 0: paper closure, 1: cubic-exact closure
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

// Cell values are stored at cv[c + CV_OFF] for c in [-4, N+2]: the four cells left of
// the line and the four right of it are the ones the outer ghost coefficients reach.
constexpr int CV_OFF = 4;
template <int N>
struct CellCount { static constexpr int value = N + 7; };

// Cell values of one line, handed out as soon as each patch is solved:
// emit(std::integral_constant<int, c>{}, value) for c in [-4, N+2].  Emitting early
// keeps only one patch's coefficients live at a time.
template <typename T, int N, int M, int G, typename Ptr, typename Emit>
__host__ __device__ __forceinline__ void line_emit(const T (&v)[N], const AxisCoef<T, Ptr>& k, Emit&& emit)
{
    using S = Shape<N, M>;
    constexpr int P = S::P;
    constexpr int W = 2 * G + 1;
    constexpr int MF = M + 1;

    // 1. interface slopes
    T d[P + 1];
    static_for<0, P + 1>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int I = S::iface(q);
        T acc = T(0);
        static_for<0, W>([&](auto tc) {
            constexpr int j = I - G + decltype(tc)::value;
            if constexpr (j >= 0 && j < N) acc = fma(k.stencil[q * W + decltype(tc)::value], v[j], acc);
        });
        d[q] = acc;
    });

    static_for<0, P>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        constexpr int s = S::start(l);
        constexpr int m = S::cells(l);
        const Ptr f = k.fac + (l == P - 1 ? 3 * MF : 0);
        const Ptr inv = f;
        const Ptr ainv = f + MF;
        const Ptr cp = f + 2 * MF;

        // 2. forward sweep of the reduced tridiagonal system
        T e[m + 1];
        e[0] = fma(k.h3, d[l], v[s]) * inv[0];
        static_for<1, m + 1>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            T r = v[s + i];
            if constexpr (i == m) r = fma(-k.h3, d[l + 1], r);
            e[i] = fma(-ainv[i], e[i - 1], r * inv[i]);
        });
        // back substitution: eta[u] = eta_{u-1}, u = 0..m+2
        T eta[m + 3];
        eta[m + 1] = e[m];
        static_for<0, m>([&](auto ic) {
            constexpr int i = m - 1 - decltype(ic)::value;
            eta[i + 1] = fma(-cp[i], eta[i + 2], e[i]);
        });
        eta[0] = fma(-k.twoh, d[l], eta[2]);
        eta[m + 2] = fma(k.twoh, d[l + 1], eta[m]);

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
            // beyond the left end: eta_{-2} is the ghost, further out zero
            const T gl = k.ghost * (4 * eta[0] - 6 * eta[1] + 4 * eta[2] - eta[3]);
            emit(std::integral_constant<int, -1>{}, fma(k.w3, eta[2], fma(k.w2, eta[1], fma(k.w1, eta[0], k.w0 * gl))));
            emit(std::integral_constant<int, -2>{}, fma(k.w3, eta[1], fma(k.w2, eta[0], k.w1 * gl)));
            emit(std::integral_constant<int, -3>{}, fma(k.w3, eta[0], k.w2 * gl));
            emit(std::integral_constant<int, -4>{}, k.w3 * gl);
        }
        if constexpr (l == P - 1) {
            // beyond the right end: eta_{m+2} is the ghost
            const T gr = k.ghost * (4 * eta[m + 2] - 6 * eta[m + 1] + 4 * eta[m] - eta[m - 1]);
            emit(std::integral_constant<int, N - 1>{},
                 fma(k.w3, gr, fma(k.w2, eta[m + 2], fma(k.w1, eta[m + 1], k.w0 * eta[m]))));
            emit(std::integral_constant<int, N>{}, fma(k.w2, gr, fma(k.w1, eta[m + 2], k.w0 * eta[m + 1])));
            emit(std::integral_constant<int, N + 1>{}, fma(k.w1, gr, k.w0 * eta[m + 2]));
            emit(std::integral_constant<int, N + 2>{}, k.w0 * gr);
        }
    });
}

// Cell values of one line.  v[N] in, cv[c + CV_OFF] out for c in [-4, N+2].
template <typename T, int N, int M, int G, typename Ptr>
__host__ __device__ __forceinline__ void line_cells(const T (&v)[N], T (&cv)[N + 7], const AxisCoef<T, Ptr>& k)
{
    line_emit<T, N, M, G>(v, k, [&](auto cc, T x) { cv[decltype(cc)::value + CV_OFF] = x; });
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
// output node j = c - SIG as soon as its patch is solved; SIG_ANY collects the cell
// values and moves them through the barrel shifter.
template <typename T, int N, int M, int G, int SIG, typename Ptr, typename Store>
__host__ __device__ __forceinline__ void advect_line(const T (&v)[N], const AxisCoef<T, Ptr>& k, int sigma, Store st)
{
    if constexpr (SIG == 0 || SIG == -1) {
        line_emit<T, N, M, G>(v, k, [&](auto cc, T x) {
            constexpr int j = decltype(cc)::value - SIG;
            if constexpr (j >= 0 && j < N) st(j, x);
        });
    } else {
        T cv[N + 7];
        line_cells<T, N, M, G>(v, cv, k);
        store_cells<T, N, SIG_ANY>(cv, sigma, st);
    }
}

// Convenience form with the dispatch inside (one line; used off the hot loops).
template <typename T, int N, typename Store>
__host__ __device__ __forceinline__ void store_shifted(const T (&cv)[N + 7], int sigma, Store st)
{
    dispatch_sigma(sigma, [&](auto sc) { store_cells<T, N, decltype(sc)::value>(cv, sigma, st); });
}

}  // namespace chasm

// chasm_ho2d.hip -- the 2-D harmonic-oscillator workload of Sec. 5.1 (see
// include/chasm_ho2d.h): LPC1 with the patched-spline characteristic step in x and the
// spectral k-derivative Theta[f] = omega x d_k f, all FP64.
//
// Kernels:
//   k_ho_advect  the characteristic step of LB k-lines per block, lines of runtime
//                length in LDS: PMBC interface slopes (eqs. 3.4-3.5), each patch's
//                reduced Hermite system solved as a product with its precomputed
//                inverse (one output per thread, so a line's patches solve in parallel),
//                the Hermite ghosts, and the 4-tap evaluation by the owning patch
//                (eqs. 3.7-3.8, Sec. 3.1.3), out of place; departure points outside
//                the line give 0 unless the descriptor asks for ghost extrapolation.
//   k_ho_dk      Theta by transforms, for nk = L1 L2 a power of two in 64..1024: two
//                real k-lines (x columns 2c, 2c+1) form one complex line, since the
//                derivative F^-1 diag(i xi) F maps real lines to real lines; a
//                four-step transform (L1-point register transforms over stride-L2
//                elements, twiddles, L2-point register transforms), the multiply by
//                i xi / nk (Nyquist mode 0) and the inverse in reverse order, with two
//                LDS transposes per line.  Mode 1 fuses the LPC1 corrector: it reads
//                FA, GA, transforms Y = FA + tau GA and writes FA + tau/2 (GA + Theta Y).
//   k_ho_dk512   nk = 512: the same transform pair in three levels of 8-point
//                transforms, one complex line per 64-thread block.
//   k_ho_theta   any other even nk: out[k][x] = omega x sum_q D[k][q] f[q][x], a dense
//                FP64 contraction with the circulant spectral differentiation matrix,
//                32 x 32 output tiles staged through LDS, 2 x 2 outputs per thread.
//   k_ho_combine the predictor / corrector combinations of the dense path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/chasm_ho2d.h"
#include "chasm_fft.hpp"
#include "chasm_tables.hpp"

namespace chasm {
void set_last_error(const std::string& msg);

struct HoArgs {
    int N, M, P, mlast, g, nk, inflow;
    double hx;
    const double* stencil;     // (P+1) x (2g+1), slopes (not times h)
    const double* ainvM;       // (M+1)^2 inverse of [4 2; 1 4 1; ...; 2 4]
    const double* ainvL;       // (mlast+1)^2
    const int* shift;          // nk
    const double* w;           // nk x 4
};

constexpr int HO_LB = 2;       // lines per block (measured at nx = 241, 1024 lines: 8 -> 21.5 us, 4 -> 15.7, 2 -> 14.7)

__global__ __launch_bounds__(256) void k_ho_advect(const double* __restrict__ in, double* __restrict__ out, const HoArgs a,
                                                  int nlines)
{
    extern __shared__ double sm[];
    const int N = a.N, M = a.M, P = a.P;
    const int ES = N - 1 + 3 * P;                    // sum over patches of (m + 3)
    double* phi = sm;                                // [LB][N]
    double* dsl = phi + HO_LB * N;                   // [LB][P+1] slopes times h
    double* eta = dsl + HO_LB * (P + 1);             // [LB][ES], patch l at l (M+3): eta_{-1..m+1}
    const int line0 = blockIdx.x * HO_LB;
    const int tid = threadIdx.x;

    for (int e = tid; e < HO_LB * N; e += blockDim.x) {
        const int ln = e / N, L = line0 + ln;
        phi[e] = L < nlines ? in[(long long)L * N + e % N] : 0.0;
    }
    __syncthreads();
    const int W = 2 * a.g + 1;
    for (int e = tid; e < HO_LB * (P + 1); e += blockDim.x) {
        const int ln = e / (P + 1), q = e % (P + 1);
        const int I = q < P ? q * M : N - 1;
        double acc = 0.0;
        for (int t = 0; t < W; ++t) {
            const int j = I - a.g + t;
            if (j >= 0 && j < N) acc = fma(a.stencil[q * W + t], phi[ln * N + j], acc);
        }
        dsl[e] = acc * a.hx;
    }
    __syncthreads();
    // each thread takes one row i of one patch's inverse and applies it to the right-hand
    // sides of all LB lines: rhs_jj = 6 phi_jj, plus 2 h d_L at jj = 0 and minus 2 h d_R at
    // jj = m (added after the loop, the product being linear)
    const int per_line = N - 1 + P;                  // unknowns eta_0..eta_m of every patch
    for (int r = tid; r < per_line; r += blockDim.x) {
        const int l = min(r / (M + 1), P - 1);
        const int i = r - l * (M + 1);
        const int m = l < P - 1 ? M : a.mlast;
        const double* A = (l < P - 1 ? a.ainvM : a.ainvL) + (long long)i * (m + 1);
        double acc[HO_LB];
#pragma unroll
        for (int ln = 0; ln < HO_LB; ++ln) acc[ln] = 0.0;
        for (int jj = 0; jj <= m; ++jj) {
            const double aij = 6.0 * A[jj];
#pragma unroll
            for (int ln = 0; ln < HO_LB; ++ln) acc[ln] = fma(aij, phi[ln * N + l * M + jj], acc[ln]);
        }
        const double a0 = 2.0 * A[0], am = 2.0 * A[m];
#pragma unroll
        for (int ln = 0; ln < HO_LB; ++ln)
            eta[ln * ES + l * (M + 3) + 1 + i] =
                acc[ln] + a0 * dsl[ln * (P + 1) + l] - am * dsl[ln * (P + 1) + l + 1];
    }
    __syncthreads();
    for (int e = tid; e < HO_LB * P; e += blockDim.x) {
        const int ln = e / P, l = e % P;
        const int m = l < P - 1 ? M : a.mlast;
        double* E = eta + ln * ES + l * (M + 3);
        E[0] = E[2] - 2.0 * dsl[ln * (P + 1) + l];                // eta_{-1} = eta_1 - 2 h d_L
        E[m + 2] = E[m] + 2.0 * dsl[ln * (P + 1) + l + 1];        // eta_{m+1} = eta_{m-1} + 2 h d_R
    }
    __syncthreads();
    for (int e = tid; e < HO_LB * N; e += blockDim.x) {
        const int ln = e / N, j = e % N, L = line0 + ln;
        if (L >= nlines) continue;
        const int kk = L % a.nk;
        const int c = j + a.shift[kk];                           // departure cell
        double v = 0.0;
        // departure point inside [x_0, x_{N-1}]: cell 0 .. N-2, or exactly node N-1
        // (beta = 0, i.e. w3 = beta^3/6 = 0)
        const bool inside = c >= 0 && (c < N - 1 || (c == N - 1 && a.w[4 * kk + 3] == 0.0));
        if ((inside || a.inflow == 1) && c >= -4 && c <= N + 2) {
            const int l = c < 0 ? 0 : min(c / M, P - 1);         // owner patch
            const int m = l < P - 1 ? M : a.mlast;
            const int nu = c - l * M;
            const double* E = eta + ln * ES + l * (M + 3);
            const double* w = a.w + 4 * kk;
            for (int r = 0; r < 4; ++r) {
                const int u = nu - 1 + r;                        // eta_u, zero beyond the ghosts
                if (u >= -1 && u <= m + 1) v = fma(w[r], E[u + 1], v);
            }
        }
        out[(long long)L * N + j] = v;
    }
}

__global__ __launch_bounds__(256) void k_ho_theta(const double* __restrict__ D, const double* __restrict__ f,
                                                 double* __restrict__ out, int nk, int nx, double x_lo, double hx,
                                                 double omega)
{
    // 32 x 32 output tile per block (2 x 2 per thread), k-chunks of 32 through LDS
    __shared__ double As[32][33];                       // As[q][r] = D[r0 + r][q0 + q]
    __shared__ double Bs[32][33];                       // Bs[q][c] = f[q0 + q][c0 + c]
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    double acc[2][2] = {};
    for (int q0 = 0; q0 < nk; q0 += 32) {
        for (int e = threadIdx.x; e < 32 * 32; e += 256) {
            const int rr = e / 32, qq = e % 32;
            const int r = r0 + rr, q = q0 + qq;
            As[qq][rr] = (r < nk && q < nk) ? D[(long long)r * nk + q] : 0.0;
            const int qb = e / 32, cc = e % 32;
            const int qf = q0 + qb, x = c0 + cc;
            Bs[qb][cc] = (qf < nk && x < nx) ? f[(long long)qf * nx + x] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int qq = 0; qq < 32; ++qq) {
            const double a0 = As[qq][ty], a1 = As[qq][ty + 16];
            const double b0 = Bs[qq][tx], b1 = Bs[qq][tx + 16];
            acc[0][0] = fma(a0, b0, acc[0][0]);
            acc[0][1] = fma(a0, b1, acc[0][1]);
            acc[1][0] = fma(a1, b0, acc[1][0]);
            acc[1][1] = fma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i) {
        const int r = r0 + ty + 16 * i;
        if (r >= nk) continue;
        for (int j = 0; j < 2; ++j) {
            const int x = c0 + tx + 16 * j;
            if (x < nx) out[(long long)r * nx + x] = omega * (x_lo + x * hx) * acc[i][j];
        }
    }
}

struct DkArgs {
    int nx;
    double x_lo, hx, hk, omega, tau;
};

// Complex lines per block and threads per block of k_ho_dk (one wave).
template <int L1, int L2>
struct DkShape {
    static constexpr int L = L1 * L2;
    static constexpr int TL = L2 > L1 ? L2 : L1;     // threads per complex line
    static constexpr int CLB = 64 / TL;              // complex lines per block
    static constexpr int NT = CLB * TL;
    static constexpr int RS = L2 + 1;                // LDS row of [k1][n2], padded
};

// MODE 0: out = omega x d_k a.  MODE 1: y = a + tau b, out = (a + tau/2 b) + tau/2 omega x d_k y.
// tw[j] = e^{+2 pi i j / L}.  Index convention of the four-step transform: element
// n = L2 n1 + n2, frequency m = k1 + L1 k2.  Each lane reads and writes its own
// elements in HBM (one wave per block, so the block count, not the run length of a
// row, sets how much of the chip takes part: staging a 16-column tile through LDS
// for row-contiguous accesses ran 2.3x slower at nx = 241, nk = 512).
template <int L1, int L2, int MODE>
__global__ __launch_bounds__(64) void k_ho_dk(const double* __restrict__ a, const double* __restrict__ b,
                                              double* __restrict__ out, const fft::cd* __restrict__ tw,
                                              const DkArgs p)
{
    using namespace fft;
    using S = DkShape<L1, L2>;
    static_assert(S::NT == 64, "one wave per block");
    constexpr int L = S::L;
    __shared__ cd lds[S::CLB * L1 * S::RS];
    const int lt = threadIdx.x % S::TL, cl = threadIdx.x / S::TL;
    const int xa = 2 * (blockIdx.x * S::CLB + cl), xb = xa + 1;
    const bool has_a = xa < p.nx, has_b = xb < p.nx;
    cd* Y = lds + cl * L1 * S::RS;

    // MODE 1 keeps a + tau/2 b of the thread's output elements from step 1 to step 3
    // (the same rows and columns), so step 3 issues no dependent loads.
    const double h = 0.5 * p.tau;
    cd keep[MODE == 1 ? L1 : 1];
    // Step 1 (thread n2 = lt): L1-point transforms over n1, twiddle e^{-2 pi i n2 k1 / L}.
    if (lt < L2 && has_a) {
        const int n2 = lt;
        cd v[L1];
        sfor<0, L1>([&](auto ic) {
            constexpr int n1 = decltype(ic)::value;
            const long long row = (long long)(L2 * n1 + n2) * p.nx;
            if constexpr (MODE == 0) {
                v[n1] = {a[row + xa], has_b ? a[row + xb] : 0.0};
            } else {
                const double aa = a[row + xa], ba = b[row + xa];
                const double ab = has_b ? a[row + xb] : 0.0, bb = has_b ? b[row + xb] : 0.0;
                v[n1] = {fma(p.tau, ba, aa), fma(p.tau, bb, ab)};
                keep[n1] = {fma(h, ba, aa), fma(h, bb, ab)};
            }
        });
        transform<L1, -1>(v);
        sfor<0, L1>([&](auto kc) {
            constexpr int k1 = decltype(kc)::value;
            cd w = v[k1];
            if constexpr (k1 > 0) w = cmul(w, conj(tw[(n2 * k1) & (L - 1)]));
            Y[k1 * S::RS + n2] = w;
        });
    }
    __syncthreads();
    // Step 2 (thread k1 = lt): L2-point transforms over n2 give X[k1 + L1 k2]; multiply by
    // i xi_m / L; inverse L2-point transforms; twiddle e^{+2 pi i n2 k1 / L}.
    if (lt < L1 && has_a) {
        const int k1 = lt;
        cd v[L2];
        sfor<0, L2>([&](auto ic) { v[decltype(ic)::value] = Y[k1 * S::RS + decltype(ic)::value]; });
        transform<L2, -1>(v);
        const double unit = 2.0 * kPi / (L * p.hk) / L;
        sfor<0, L2>([&](auto kc) {
            constexpr int k2 = decltype(kc)::value;
            const int m = k1 + L1 * k2;
            const double xi = m < L / 2 ? (double)m * unit : (m == L / 2 ? 0.0 : (double)(m - L) * unit);
            v[k2] = {-xi * v[k2].im, xi * v[k2].re};
        });
        transform<L2, +1>(v);
        sfor<0, L2>([&](auto nc) {
            constexpr int n2 = decltype(nc)::value;
            cd w = v[n2];
            if constexpr (n2 > 0) w = cmul(w, tw[(n2 * k1) & (L - 1)]);
            Y[k1 * S::RS + n2] = w;
        });
    }
    __syncthreads();
    // Step 3 (thread n2 = lt): inverse L1-point transforms over k1 give d_k y at rows
    // L2 n1 + n2; real part column xa, imaginary part column xb.
    if (lt < L2 && has_a) {
        const int n2 = lt;
        cd v[L1];
        sfor<0, L1>([&](auto kc) { v[decltype(kc)::value] = Y[decltype(kc)::value * S::RS + n2]; });
        transform<L1, +1>(v);
        const double fa = p.omega * (p.x_lo + xa * p.hx), fb = p.omega * (p.x_lo + xb * p.hx);
        sfor<0, L1>([&](auto ic) {
            constexpr int n1 = decltype(ic)::value;
            const long long row = (long long)(L2 * n1 + n2) * p.nx;
            if constexpr (MODE == 0) {
                out[row + xa] = fa * v[n1].re;
                if (has_b) out[row + xb] = fb * v[n1].im;
            } else {
                out[row + xa] = fma(h, fa * v[n1].re, keep[n1].re);
                if (has_b) out[row + xb] = fma(h, fb * v[n1].im, keep[n1].im);
            }
        });
    }
}

// nk = 512 = 8 x 8 x 8: a three-level form of the same transform pair, so that every
// thread's serial chain is six 8-point transforms (the four-step form above runs two
// 32-point transforms per thread in its middle step).  One complex line (x columns 2c,
// 2c+1) per 64-thread block.  Index convention: element n = 64 n1 + 8 n2 + n3,
// frequency m = m1 + 8 m2 + 64 m3;
//   step 1   (n2, n3): 8-point transform over n1, twiddle e^{-2 pi i (8 n2 + n3) m1 / 512}
//   step 2   (m1, n3): 8-point transform over n2, twiddle e^{-2 pi i 8 n3 m2 / 512}
//   step 3   (m1, m2): 8-point transform over n3, times i xi_m / 512, inverse over m3
//   steps 2', 1': the inverses of steps 2 and 1 with conjugate twiddles.
template <int MODE>
__global__ __launch_bounds__(64) void k_ho_dk512(const double* __restrict__ a, const double* __restrict__ b,
                                                double* __restrict__ out, const fft::cd* __restrict__ tw,
                                                const DkArgs p)
{
    using namespace fft;
    constexpr int L = 512, RS = 65;                 // LDS rows of 64 values, padded
    __shared__ cd S1[8 * RS];                        // [m1][n3][n2]
    __shared__ cd S2[8 * RS];                        // [m1][m2][n3]
    const int t = threadIdx.x, lo = t & 7, hi = t >> 3;
    const int xa = 2 * blockIdx.x, xb = xa + 1;
    const bool has_b = xb < p.nx;
    const double h = 0.5 * p.tau;
    cd v[8];
    cd keep[MODE == 1 ? 8 : 1];
    // step 1: (n2, n3) = (lo, hi)
    sfor<0, 8>([&](auto ic) {
        constexpr int n1 = decltype(ic)::value;
        const long long row = (long long)(64 * n1 + 8 * lo + hi) * p.nx;
        if constexpr (MODE == 0) {
            v[n1] = {a[row + xa], has_b ? a[row + xb] : 0.0};
        } else {
            const double aa = a[row + xa], ba = b[row + xa];
            const double ab = has_b ? a[row + xb] : 0.0, bb = has_b ? b[row + xb] : 0.0;
            v[n1] = {fma(p.tau, ba, aa), fma(p.tau, bb, ab)};
            keep[n1] = {fma(h, ba, aa), fma(h, bb, ab)};
        }
    });
    transform<8, -1>(v);
    sfor<0, 8>([&](auto mc) {
        constexpr int m1 = decltype(mc)::value;
        cd w = v[m1];
        if constexpr (m1 > 0) w = cmul(w, conj(tw[((8 * lo + hi) * m1) & (L - 1)]));
        S1[m1 * RS + 8 * hi + lo] = w;
    });
    __syncthreads();
    // step 2: (m1, n3) = (lo, hi)
    sfor<0, 8>([&](auto ic) { v[decltype(ic)::value] = S1[lo * RS + 8 * hi + decltype(ic)::value]; });
    transform<8, -1>(v);
    sfor<0, 8>([&](auto mc) {
        constexpr int m2 = decltype(mc)::value;
        cd w = v[m2];
        if constexpr (m2 > 0) w = cmul(w, conj(tw[(8 * hi * m2) & (L - 1)]));
        S2[lo * RS + 8 * m2 + hi] = w;
    });
    __syncthreads();
    // step 3: (m1, m2) = (lo, hi); the row is this thread's alone, read and written back
    sfor<0, 8>([&](auto ic) { v[decltype(ic)::value] = S2[lo * RS + 8 * hi + decltype(ic)::value]; });
    transform<8, -1>(v);
    const double unit = 2.0 * kPi / (L * p.hk) / L;
    sfor<0, 8>([&](auto mc) {
        constexpr int m3 = decltype(mc)::value;
        const int m = lo + 8 * hi + 64 * m3;
        const double xi = m < L / 2 ? (double)m * unit : (m == L / 2 ? 0.0 : (double)(m - L) * unit);
        v[m3] = {-xi * v[m3].im, xi * v[m3].re};
    });
    transform<8, +1>(v);
    sfor<0, 8>([&](auto ic) { S2[lo * RS + 8 * hi + decltype(ic)::value] = v[decltype(ic)::value]; });
    __syncthreads();
    // step 2': (m1, n3) = (lo, hi)
    sfor<0, 8>([&](auto mc) {
        constexpr int m2 = decltype(mc)::value;
        const cd x = S2[lo * RS + 8 * m2 + hi];
        v[m2] = m2 > 0 ? cmul(x, tw[(8 * hi * m2) & (L - 1)]) : x;
    });
    transform<8, +1>(v);
    sfor<0, 8>([&](auto ic) { S1[lo * RS + 8 * hi + decltype(ic)::value] = v[decltype(ic)::value]; });
    __syncthreads();
    // step 1': (n2, n3) = (lo, hi); d_k y at rows 64 n1 + 8 n2 + n3
    sfor<0, 8>([&](auto mc) {
        constexpr int m1 = decltype(mc)::value;
        const cd x = S1[m1 * RS + 8 * hi + lo];
        v[m1] = m1 > 0 ? cmul(x, tw[((8 * lo + hi) * m1) & (L - 1)]) : x;
    });
    transform<8, +1>(v);
    const double fa = p.omega * (p.x_lo + xa * p.hx), fb = p.omega * (p.x_lo + xb * p.hx);
    sfor<0, 8>([&](auto ic) {
        constexpr int n1 = decltype(ic)::value;
        const long long row = (long long)(64 * n1 + 8 * lo + hi) * p.nx;
        if constexpr (MODE == 0) {
            out[row + xa] = fa * v[n1].re;
            if (has_b) out[row + xb] = fb * v[n1].im;
        } else {
            out[row + xa] = fma(h, fa * v[n1].re, keep[n1].re);
            if (has_b) out[row + xb] = fma(h, fb * v[n1].im, keep[n1].im);
        }
    });
}

// mode 0: dst = a + c b;  mode 1: dst = a + c (b + y)
__global__ __launch_bounds__(256) void k_ho_combine(double* __restrict__ dst, const double* __restrict__ a,
                                                   const double* __restrict__ b, const double* __restrict__ y,
                                                   long long n, double c, int mode)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        dst[i] = mode == 0 ? fma(c, b[i], a[i]) : fma(c, b[i] + y[i], a[i]);
}

// Inverse of the (m+1) x (m+1) reduced patch matrix [4 2; 1 4 1; ...; 2 4] (the Hermite
// rows of eq. 2.13 eliminated into the interpolation rows of eq. 2.12, times 6), by
// Gauss-Jordan elimination (diagonally dominant: no pivoting needed).
static std::vector<double> patch_inverse(int m)
{
    const int n = m + 1;
    std::vector<double> A((size_t)n * n, 0.0), I((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        A[(size_t)i * n + i] = 4.0;
        if (i > 0) A[(size_t)i * n + i - 1] = i == n - 1 ? 2.0 : 1.0;
        if (i < n - 1) A[(size_t)i * n + i + 1] = i == 0 ? 2.0 : 1.0;
        I[(size_t)i * n + i] = 1.0;
    }
    for (int k = 0; k < n; ++k) {
        const double p = A[(size_t)k * n + k];
        for (int j = 0; j < n; ++j) {
            A[(size_t)k * n + j] /= p;
            I[(size_t)k * n + j] /= p;
        }
        for (int r = 0; r < n; ++r) {
            if (r == k) continue;
            const double f = A[(size_t)r * n + k];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)r * n + j] -= f * A[(size_t)k * n + j];
                I[(size_t)r * n + j] -= f * I[(size_t)k * n + j];
            }
        }
    }
    return I;
}

// Spectral differentiation on the periodic grid of n (even) points, spacing h:
// D[p][q] = d(p - q), d(0) = 0, d(r) = (pi / (n h)) (-1)^r cot(pi r / n) -- the matrix of
// F^-1 diag(i xi) F with the Nyquist mode's derivative set to zero.
static std::vector<double> spectral_dk(int n, double h)
{
    std::vector<double> d(n, 0.0), D((size_t)n * n);
    for (int r = 1; r < n; ++r) d[r] = (M_PI / (n * h)) * ((r % 2) ? -1.0 : 1.0) / std::tan(M_PI * r / n);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) D[(size_t)p * n + q] = d[((p - q) % n + n) % n];
    return D;
}

}  // namespace chasm

using namespace chasm;

struct chasm_ho2d_s {
    chasm_ho2d_desc desc;
    hipStream_t stream = nullptr;
    HoArgs args{};
    void* tables = nullptr;
    double* D = nullptr;             // dense path: the differentiation matrix
    fft::cd* tw = nullptr;           // transform path: e^{+2 pi i j / nk}, j < nk
    double *X = nullptr, *XA = nullptr, *Y = nullptr, *Z = nullptr;   // X, XA: two fields each
    double* f = nullptr;
    long long n = 0;
    bool poisoned = false;
};

static chasm_status hfail(chasm_status st, const std::string& m)
{
    set_last_error(m);
    return st;
}

// Transform path for nk in {64, ..., 1024}: nk = L1 L2.
static bool dk_by_transform(int nk) { return nk >= 64 && nk <= 1024 && (nk & (nk - 1)) == 0; }

template <int L1, int L2>
static void launch_dk_t(int mode, const double* a, const double* b, double* out, const fft::cd* tw, const DkArgs& p,
                        hipStream_t s)
{
    using S = DkShape<L1, L2>;
    const int ncl = (p.nx + 1) / 2;
    const dim3 grid((unsigned)((ncl + S::CLB - 1) / S::CLB));
    if (mode == 0)
        hipLaunchKernelGGL((k_ho_dk<L1, L2, 0>), grid, dim3(S::NT), 0, s, a, b, out, tw, p);
    else
        hipLaunchKernelGGL((k_ho_dk<L1, L2, 1>), grid, dim3(S::NT), 0, s, a, b, out, tw, p);
}

static void launch_dk(int nk, int mode, const double* a, const double* b, double* out, const fft::cd* tw,
                      const DkArgs& p, hipStream_t s)
{
    switch (nk) {
    case 64: launch_dk_t<8, 8>(mode, a, b, out, tw, p, s); break;
    case 128: launch_dk_t<8, 16>(mode, a, b, out, tw, p, s); break;
    case 256: launch_dk_t<16, 16>(mode, a, b, out, tw, p, s); break;
    case 512: {
        const dim3 grid((unsigned)((p.nx + 1) / 2));
        if (mode == 0)
            hipLaunchKernelGGL(k_ho_dk512<0>, grid, dim3(64), 0, s, a, b, out, tw, p);
        else
            hipLaunchKernelGGL(k_ho_dk512<1>, grid, dim3(64), 0, s, a, b, out, tw, p);
        break;
    }
    default: launch_dk_t<32, 32>(mode, a, b, out, tw, p, s); break;
    }
}

extern "C" {

chasm_status chasm_ho2d_create(const chasm_ho2d_desc* d, void* f_dev, void* hip_stream, chasm_ho2d_t* out)
{
    if (!out) return hfail(CHASM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d || !f_dev) return hfail(CHASM_EINVAL, "NULL argument");
    if (d->nx < 2 || d->nx > 1024) return hfail(CHASM_EINVAL, "nx must be in 2..1024");
    if (d->nk < 2 || d->nk > 4096 || d->nk % 2) return hfail(CHASM_EINVAL, "nk must be even, 2..4096");
    if (!(d->hx > 0) || !(d->hk > 0) || !std::isfinite(d->x_lo) || !std::isfinite(d->k_lo) || !std::isfinite(d->hx) ||
        !std::isfinite(d->hk))
        return hfail(CHASM_EINVAL, "grid spacings must be finite and > 0");
    if (d->patch < 2 || d->patch > d->nx - 1) return hfail(CHASM_EINVAL, "patch must be in 2..nx-1");
    if (d->ghost < 1 || d->ghost > d->nx - 1) return hfail(CHASM_EINVAL, "ghost must be in 1..nx-1");
    if (!std::isfinite(d->omega) || !(d->tau > 0) || !std::isfinite(d->tau))
        return hfail(CHASM_EINVAL, "omega must be finite and tau finite and > 0");
    if (d->inflow != 0 && d->inflow != 1) return hfail(CHASM_EINVAL, "inflow must be 0 or 1");

    AxisTables at;
    std::string err;
    if (!build_axis_tables(d->nx, d->patch, d->ghost, d->ghost, d->hx, 0, d->nk, d->k_lo, d->hk, d->tau, at, err))
        return hfail(CHASM_EINVAL, err);
    const int P = at.P, M = d->patch, mlast = at.MLAST;
    if ((size_t)HO_LB * (2 * d->nx + 4 * P) * sizeof(double) > 65536)
        return hfail(CHASM_EINVAL, "lines too long for the LDS line kernel (2 lines of 2 nx + 4 P doubles <= 64 KiB)");
    const bool by_transform = dk_by_transform(d->nk);
    const std::vector<double> AM = patch_inverse(M), AL = patch_inverse(mlast);
    const std::vector<double> D = by_transform ? std::vector<double>() : spectral_dk(d->nk, d->hk);
    std::vector<fft::cd> TW;
    if (by_transform)
        for (int j = 0; j < d->nk; ++j) TW.push_back(fft::twiddle(j, d->nk, +1));

    chasm_ho2d_s* h = new (std::nothrow) chasm_ho2d_s();
    if (!h) return hfail(CHASM_ENOMEM, "host allocation failed");
    h->desc = *d;
    h->stream = (hipStream_t)hip_stream;
    h->f = static_cast<double*>(f_dev);
    h->n = (long long)d->nk * d->nx;
    auto bail = [&](chasm_status s, const std::string& m) {
        chasm_ho2d_destroy(h);
        return hfail(s, m);
    };
    // one block: stencil | ainvM | ainvL | w (doubles), then shift (ints)
    const size_t nd = at.stencil.size() + AM.size() + AL.size() + at.w.size();
    std::vector<char> blob(nd * sizeof(double) + at.shift.size() * sizeof(int));
    double* dp = reinterpret_cast<double*>(blob.data());
    size_t o = 0;
    const size_t o_st = o; std::copy(at.stencil.begin(), at.stencil.end(), dp + o); o += at.stencil.size();
    const size_t o_am = o; std::copy(AM.begin(), AM.end(), dp + o); o += AM.size();
    const size_t o_al = o; std::copy(AL.begin(), AL.end(), dp + o); o += AL.size();
    const size_t o_w = o; std::copy(at.w.begin(), at.w.end(), dp + o); o += at.w.size();
    std::copy(at.shift.begin(), at.shift.end(), reinterpret_cast<int*>(dp + o));
    if (hipMalloc(&h->tables, blob.size()) != hipSuccess) return bail(CHASM_ENOMEM, "hipMalloc(tables) failed");
    if (!by_transform && hipMalloc((void**)&h->D, D.size() * sizeof(double)) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(D) failed");
    if (by_transform && hipMalloc((void**)&h->tw, TW.size() * sizeof(fft::cd)) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(twiddles) failed");
    const size_t fb = (size_t)h->n * sizeof(double);
    if (hipMalloc((void**)&h->X, 2 * fb) != hipSuccess || hipMalloc((void**)&h->XA, 2 * fb) != hipSuccess ||
        hipMalloc((void**)&h->Y, fb) != hipSuccess || hipMalloc((void**)&h->Z, fb) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(state) failed");
    if (hipMemcpyAsync(h->tables, blob.data(), blob.size(), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        (h->D && hipMemcpyAsync(h->D, D.data(), D.size() * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
                     hipSuccess) ||
        (h->tw && hipMemcpyAsync(h->tw, TW.data(), TW.size() * sizeof(fft::cd), hipMemcpyHostToDevice, h->stream) !=
                      hipSuccess) ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return bail(CHASM_EDEVICE, "table upload failed");
    const double* tb = static_cast<const double*>(h->tables);
    HoArgs& a = h->args;
    a.N = d->nx;
    a.M = M;
    a.P = P;
    a.mlast = mlast;
    a.g = d->ghost;
    a.nk = d->nk;
    a.inflow = d->inflow;
    a.hx = d->hx;
    a.stencil = tb + o_st;
    a.ainvM = tb + o_am;
    a.ainvL = tb + o_al;
    a.w = tb + o_w;
    a.shift = reinterpret_cast<const int*>(tb + o);
    *out = h;
    return CHASM_OK;
}

chasm_status chasm_ho2d_step(chasm_ho2d_t h, int32_t nsteps)
{
    if (!h) return hfail(CHASM_EINVAL, "handle is NULL");
    if (h->poisoned) return hfail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    if (nsteps < 0) return hfail(CHASM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return CHASM_OK;
    const chasm_ho2d_desc& d = h->desc;
    const HoArgs& a = h->args;
    const long long n = h->n;
    const size_t fb = (size_t)n * sizeof(double);
    hipStream_t s = h->stream;
    const int nlines = 2 * d.nk;
    const size_t smem = (size_t)HO_LB * (2 * a.N + 4 * a.P) * sizeof(double);
    const dim3 tgrid((unsigned)((d.nx + 31) / 32), (unsigned)((d.nk + 31) / 32));
    const unsigned cgrid = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    double *F = h->X, *G = h->X + n, *FA = h->XA, *GA = h->XA + n;
    hipError_t e = hipMemcpyAsync(F, h->f, fb, hipMemcpyDeviceToDevice, s);
    const DkArgs dp{d.nx, d.x_lo, d.hx, d.hk, d.omega, d.tau};
    for (int it = 0; it < nsteps && e == hipSuccess && h->tw; ++it) {
        // predictor Theta F; advect (F, Theta F); corrector fused with Theta (FA + tau GA)
        launch_dk(d.nk, 0, F, nullptr, G, h->tw, dp, s);
        hipLaunchKernelGGL(k_ho_advect, dim3((unsigned)((nlines + HO_LB - 1) / HO_LB)), dim3(256), smem, s, h->X, h->XA,
                           a, nlines);
        launch_dk(d.nk, 1, FA, GA, F, h->tw, dp, s);
        e = hipGetLastError();
    }
    for (int it = 0; it < nsteps && e == hipSuccess && !h->tw; ++it) {
        hipLaunchKernelGGL(k_ho_theta, tgrid, dim3(256), 0, s, h->D, F, G, d.nk, d.nx, d.x_lo, d.hx, d.omega);
        hipLaunchKernelGGL(k_ho_advect, dim3((unsigned)((nlines + HO_LB - 1) / HO_LB)), dim3(256), smem, s, h->X, h->XA,
                           a, nlines);
        hipLaunchKernelGGL(k_ho_combine, dim3(cgrid), dim3(256), 0, s, h->Y, FA, GA, (const double*)nullptr, n, d.tau, 0);
        hipLaunchKernelGGL(k_ho_theta, tgrid, dim3(256), 0, s, h->D, h->Y, h->Z, d.nk, d.nx, d.x_lo, d.hx, d.omega);
        hipLaunchKernelGGL(k_ho_combine, dim3(cgrid), dim3(256), 0, s, F, FA, GA, h->Z, n, 0.5 * d.tau, 1);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h->f, F, fb, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
        h->poisoned = true;
        return hfail(CHASM_EDEVICE, std::string("ho2d step: ") + hipGetErrorString(e));
    }
    return CHASM_OK;
}

chasm_status chasm_ho2d_destroy(chasm_ho2d_t h)
{
    if (!h) return CHASM_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void* p : {(void*)h->tables, (void*)h->D, (void*)h->tw, (void*)h->X, (void*)h->XA, (void*)h->Y, (void*)h->Z})
        if (p) (void)hipFree(p);
    delete h;
    return CHASM_OK;
}

}  // extern "C"

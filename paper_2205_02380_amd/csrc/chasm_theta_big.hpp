// chasm_theta_big.hpp -- the truncated-kernel evaluation of Theta_V (Sec. 4, eq. 4.6
// with the tensor of eq. 4.9) for k-grids whose per-x-point intermediate does not fit
// in one CU (N_k = 32 and 64; also built for 16 to check it against the one-block form
// of chasm_theta.hpp).  Same mathematics as k_theta:
//   Theta(x, k_p) = sum_a w_a Im( e^{i phi_a.p} [circular convolution of period
//                   P = 2 N_k of T with the zero-padded e^{-i phi_a.p'} f_p'](p) ),
// evaluated in three stages over a batch of x-points, with a complex FP64
// intermediate in device memory, W[x][xi1][k3][k2]:
//   k_thA    modulate each k1 line and transform it along k1 (zero padded to P);
//   k_thBCD  per (x, xi1): transform along k2 (zero padded), the Toeplitz product
//            along k3 with K(xi1, xi2, |q3|) (the kernel transformed along k1 and k2,
//            see tensor_partial), and the inverse along k2 (first N_k outputs);
//   k_thE    inverse along k1 (first N_k outputs), demodulate, take the imaginary
//            part, accumulate over the nuclei.
// Every P-point transform of a zero-padded line, and every inverse restricted to the
// first N_k outputs, is split by residue: output (input) index S f + h, f < 32,
// h < S = P / 32, is a 32-point transform of the twiddled line folded modulo 32, so
// each work item holds 32 complex values in registers.  The field is in x-major order
// [b][x][k3][k2][k1], as for k_theta.
#pragma once
#include <hip/hip_runtime.h>

#include "chasm_fft.hpp"
#include "chasm_theta.hpp"

namespace chasm {

template <int NK>
struct BigShape {
    static constexpr int P = 2 * NK;
    static constexpr int L = 32;              // transform length of a work item
    static constexpr int S = P / L;           // residues
    static constexpr int RS = NK + 1;         // padded LDS row (complex)
    static constexpr int LPB = 64;            // k-lines per block in A and E
    static constexpr int BPX = NK * NK / LPB; // blocks per x-point in A and E
    static constexpr int NTB = 2 * NK > 64 ? 2 * NK : 64;   // threads of k_thBCD
    static_assert(P % L == 0 && NK * NK % LPB == 0, "shape");
};

// Coordinates of global x-point xp (batch members stacked) and the modulation table
// E[d][k] = e^{-i phi_d k}, phi_d = 2 (x_d - x_a,d) hk_d, of nucleus nu.
template <int NK>
__device__ __forceinline__ void big_modulation(const ThetaArgs& a, long long xp, int nu, fft::cd (*E)[NK])
{
    const long long loc = xp % a.npts;
    const int i1 = (int)(loc % a.nx[0]);
    const int i2 = (int)((loc / a.nx[0]) % a.nx[1]);
    const int i3 = (int)(loc / ((long long)a.nx[0] * a.nx[1]));
    const double xc[3] = {a.x_lo[0] + i1 * a.hx[0], a.x_lo[1] + i2 * a.hx[1], a.x_lo[2] + i3 * a.hx[2]};
    for (int t = threadIdx.x; t < 3 * NK; t += blockDim.x) {
        const int d = t / NK, k = t % NK;
        const double ph = 2.0 * (xc[d] - a.xa[nu][d]) * a.hk[d] * k;
        double s, c;
        sincos(ph, &s, &c);
        E[d][k] = fft::cd{c, -s};
    }
}

// ---- A: k1 forward.  Block = 64 k1 lines of one x-point, a thread per line.
template <typename T, int NK>
__global__ __launch_bounds__(64) void k_thA(const T* __restrict__ fx, fft::cd* __restrict__ W, const ThetaArgs a,
                                            long long x0, int nu)
{
    using namespace fft;
    using B = BigShape<NK>;
    constexpr int P = B::P, S = B::S;
    __shared__ cd E[3][NK];
    const long long xl = blockIdx.x / B::BPX;
    const int la = (int)(blockIdx.x % B::BPX) * B::LPB + threadIdx.x;   // k3 * NK + k2
    const int k2 = la % NK, k3 = la / NK;
    big_modulation<NK>(a, x0 + xl, nu, E);
    __syncthreads();
    const T* line = fx + (x0 + xl) * (long long)(NK * NK * NK) + (long long)la * NK;
    const cd e23 = cmul(E[1][k2], E[2][k3]);
    cd* out = W + xl * (long long)(P * NK * NK) + la;
    sfor<0, S>([&](auto hc) {
        constexpr int h = decltype(hc)::value;
        cd y[32];
        sfor<0, 32>([&](auto jc) { y[decltype(jc)::value] = cd{0.0, 0.0}; });
        // y[k mod 32] += e^{-i phi.p} f(p) w_P^{-h k}, k = k1 < NK (zero padded to P)
        sfor<0, NK>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const double fv = (double)line[k];
            const cd e = cmul(E[0][k], e23);
            const cd z = tmul<(long long)h * k, P, -1>(cd{e.re * fv, e.im * fv});
            y[k % 32] = cadd(y[k % 32], z);
        });
        transform<32, -1>(y);
        sfor<0, 32>([&](auto fc) {
            constexpr int f = decltype(fc)::value;
            out[(long long)(S * f + h) * (NK * NK)] = y[f];   // xi1 = S f + h
        });
    });
}

// ---- B, C, D: one block per (x-point, xi1) slice W[x][xi1][k3][k2] (in place).
template <int NK>
__global__ __launch_bounds__(BigShape<NK>::NTB) void k_thBCD(fft::cd* __restrict__ W, const double* __restrict__ kt)
{
    using namespace fft;
    using B = BigShape<NK>;
    constexpr int P = B::P, L = B::L, S = B::S, RS = B::RS, NT = B::NTB;
    constexpr int JC = NK / 16;                 // 16-output chunks of a Toeplitz row
    // N_k = 32: the sum over residues stays in the registers of the thread that owns its
    // output row j3, and the kernel values K are read from the table (it sits in L2),
    // so a block needs 34 KB of LDS and four blocks (one wave per SIMD) share a CU;
    // larger N_k keep the sum and K in LDS.
    constexpr bool ACC_REG = NK == 32;
    __shared__ cd ACC[ACC_REG ? 1 : NK * RS];   // [j3][j2]: k2 inverse, summed over residues
    __shared__ cd BC[L * RS];                   // [f][k3]: k2 forward of residue h
    __shared__ cd OC[L * RS];                   // [f][j3]: after the k3 Toeplitz product
    __shared__ double KK[ACC_REG ? 1 : L * RS]; // [f][q3]: K(xi1, S f + h, q3)
    const long long xl = blockIdx.x / P;
    const int xi1 = (int)(blockIdx.x % P);
    cd* slice = W + (xl * P + xi1) * (long long)(NK * NK);
    const int tid = threadIdx.x;
    cd acc[ACC_REG ? NK : 1];                   // row j3 = tid of the residue sum (ACC_REG)

    sfor<0, S>([&](auto hc) {
        constexpr int h = decltype(hc)::value;
        // B: the k2 forward transform of every k3 row, outputs xi2 = S f + h
        for (int r = tid; r < NK; r += NT) {
            cd y[32];
            sfor<0, 32>([&](auto jc) { y[decltype(jc)::value] = cd{0.0, 0.0}; });
            const cd* row = slice + (long long)r * NK;
            sfor<0, NK>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                y[k % 32] = cadd(y[k % 32], tmul<(long long)h * k, P, -1>(row[k]));
            });
            transform<32, -1>(y);
            sfor<0, 32>([&](auto fc) { BC[decltype(fc)::value * RS + r] = y[decltype(fc)::value]; });
        }
        if constexpr (!ACC_REG) {
            for (int t = tid; t < L * NK; t += NT) {
                const int f = t / NK, q = t % NK;
                KK[f * RS + q] = kt[((long long)xi1 * P + (S * f + h)) * NK + q];
            }
        }
        __syncthreads();
        // C: o_j = sum_i K(|j - i|) row_i for each row f, 16 outputs per work item;
        // the 16 kernel values of one input form a window that slides down by one
        for (int t = tid; t < L * JC; t += NT) {
            const int f = t % L, j0 = (t / L) * 16;
            const double* kk = ACC_REG ? kt + ((long long)xi1 * P + (S * f + h)) * NK : KK + f * RS;
            const cd* row = BC + f * RS;
            cd o[16];
            double w[16];
            sfor<0, 16>([&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                o[jj] = cd{0.0, 0.0};
                w[jj] = kk[j0 + jj];            // window of input i = 0: K(|j0 + jj - 0|)
            });
            sfor<0, NK>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const cd r = row[i];
                sfor<0, 16>([&](auto jc) {
                    constexpr int jj = decltype(jc)::value;
                    o[jj].re = fma(w[jj], r.re, o[jj].re);
                    o[jj].im = fma(w[jj], r.im, o[jj].im);
                });
                if constexpr (i + 1 < NK) {
                    // window of input i + 1: K(|j0 + jj - i - 1|) = previous window shifted
                    sfor<0, 15>([&](auto jc) {
                        constexpr int jj = 15 - decltype(jc)::value;
                        w[jj] = w[jj - 1];
                    });
                    const int m = j0 - i - 1;
                    w[0] = kk[m < 0 ? -m : m];
                }
            });
            sfor<0, 16>([&](auto jc) { OC[f * RS + j0 + decltype(jc)::value] = o[decltype(jc)::value]; });
        }
        __syncthreads();
        // D: inverse along k2 over this residue's xi2, first NK outputs, summed over the
        // residues (in ACC, or in the registers of thread j3)
        for (int j3 = tid; j3 < NK; j3 += NT) {
            cd v[32];
            sfor<0, 32>([&](auto fc) { v[decltype(fc)::value] = OC[decltype(fc)::value * RS + j3]; });
            transform<32, +1>(v);
            sfor<0, NK>([&](auto jc) {
                constexpr int j2 = decltype(jc)::value;
                const cd x = tmul<(long long)h * j2, P, +1>(v[j2 % 32]);
                if constexpr (ACC_REG)
                    acc[j2] = h == 0 ? x : cadd(acc[j2], x);
                else
                    ACC[j3 * RS + j2] = h == 0 ? x : cadd(ACC[j3 * RS + j2], x);
            });
        }
        __syncthreads();
    });
    if constexpr (ACC_REG) {
        static_assert(!ACC_REG || NT >= NK, "one thread per output row");
        if (tid < NK) sfor<0, NK>([&](auto jc) { slice[tid * NK + decltype(jc)::value] = acc[decltype(jc)::value]; });
    } else {
        for (int t = tid; t < NK * NK; t += NT) {
            const int j3 = t / NK, j2 = t % NK;
            slice[t] = ACC[j3 * RS + j2];
        }
    }
}

// ---- E: k1 inverse, demodulation, imaginary part, sum over nuclei.  Block = 64 k1
// lines of one x-point.  first: no earlier nucleus; last: write the result (type T)
// to fx, else keep the FP64 sum in acc.
template <typename T, int NK>
__global__ __launch_bounds__(64) void k_thE(const fft::cd* __restrict__ W, double* __restrict__ acc,
                                            T* __restrict__ fx, const ThetaArgs a, long long x0, int nu, int first,
                                            int last)
{
    using namespace fft;
    using B = BigShape<NK>;
    constexpr int P = B::P, S = B::S, RS = B::RS;
    __shared__ cd E[3][NK];
    __shared__ double TH[B::LPB * RS];
    const long long xl = blockIdx.x / B::BPX;
    const int la = (int)(blockIdx.x % B::BPX) * B::LPB + threadIdx.x;   // j3 * NK + j2
    const int j2 = la % NK, j3 = la / NK;
    big_modulation<NK>(a, x0 + xl, nu, E);
    __syncthreads();
    const double w = a.wgt[nu];
    const cd e23c = conj(cmul(E[1][j2], E[2][j3]));
    const cd* src = W + xl * (long long)(P * NK * NK) + la;
    double* th = TH + threadIdx.x * RS;
    sfor<0, S>([&](auto hc) {
        constexpr int h = decltype(hc)::value;
        cd v[32];
        sfor<0, 32>([&](auto fc) {
            constexpr int f = decltype(fc)::value;
            v[f] = src[(long long)(S * f + h) * (NK * NK)];
        });
        transform<32, +1>(v);
        sfor<0, NK>([&](auto jc) {
            constexpr int j1 = decltype(jc)::value;
            const cd d = cmul(conj(E[0][j1]), e23c);                    // e^{+i phi.p}
            const cd t = cmul(d, tmul<(long long)h * j1, P, +1>(v[j1 % 32]));
            th[j1] = (h == 0 ? 0.0 : th[j1]) + w * t.im;
        });
    });
    const long long off = (x0 + xl) * (long long)(NK * NK * NK) + (long long)la * NK;
    double* ac = acc + xl * (long long)(NK * NK * NK) + (long long)la * NK;
    for (int j1 = 0; j1 < NK; ++j1) {
        const double v = th[j1] + (first ? 0.0 : ac[j1]);
        if (last) fx[off + j1] = (T)v;
        else ac[j1] = v;
    }
}

}  // namespace chasm

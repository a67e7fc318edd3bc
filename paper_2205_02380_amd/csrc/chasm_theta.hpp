// chasm_theta.hpp -- kernels of the truncated-kernel evaluation of the Coulomb
// pseudo-differential operator Theta_V (Sec. 4, eq. 4.6 with the tensor of eq. 4.9).
//
// At one x the operator is a discrete convolution over the N_k^3 k-grid,
//   Theta(x, k_p) = sum_a z_a (2/pi^2) Im( e^{i phi_a.p} sum_p' T_{p-p'} e^{-i phi_a.p'} f_p' ),
//   phi_a,d = 2 (x_d - x_a,d) hk_d,
// which is 2 Re of the I+ term of eq. 4.2 (the I- term is minus its conjugate for real
// f; 2/(c_{3,1} i) with c_{3,1} = 2 pi^2).  The aperiodic convolution with the
// (2N_k - 1)^3 tensor T is a circular one of period P = 2 N_k per axis: forward
// transform of the zero-padded modulated data, multiplication by That (the P^3
// transform of T, real because T is real and even), inverse transform, the first N_k
// outputs per axis.  Along k3 the transform, multiply and inverse are replaced by the
// equivalent Toeplitz product (stage C below).
//
// One x-point per block at a time (persistent over x-points), FP64 throughout.  The
// P x P x N_k intermediate of an x-point does not fit in LDS for N_k = 16 in FP64, so
// the xi1 axis is split by residue: chunk r holds xi1 = r + R m (m < C = P/R); within a
// chunk the k1 transform is a C-point DFT of folded, twiddled data (the decimation-
// in-frequency split of the P-point transform), and the k1 inverse of the chunk adds a
// C-point inverse DFT, twiddled, into the accumulator.  Stages per chunk:
//   A  k1 forward for every (k2, k3) line          -> W1[m][k3][k2]
//   B  k2 forward (zero-padded, P outputs)          -> W2[m][xi2][k3]
//   C  k3 convolution (in place): the first N_k outputs of the period-P circular
//      convolution of a zero-padded line are the Toeplitz product with the kernel
//      transformed along k1 and k2 only, K(xi1, xi2, |q3|), q3 < N_k -- the same result
//      as transform, multiply by That, inverse, in 2 N_k^2 real multiply-adds per line
//      instead of four N_k-point transforms
//   D  k2 inverse, first N_k outputs                -> W1[m][k3][k2] + W1o[m][k3][k2]
//   E  k1 inverse of the chunk, into the accumulator of each (k2, k3) line
// Rows of W1 and W2 are padded to N_k + 1 complex values, so the row-per-lane stages
// (B reads, C, D writes) and the column-per-lane stages (A, B writes, D reads, E) are
// free of LDS bank conflicts.
//
// The field is read and written in x-major order [b][x3][x2][x1][k3][k2][k1]; the
// transposes to and from the field layout are the kernels at the end of this file.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "chasm_fft.hpp"

namespace chasm {

constexpr int kMaxNuc = 4;

struct ThetaArgs {
    long long npts;              // x-points per batch member
    int nx[3];
    int nnuc;
    double x_lo[3], hx[3], hk[3];
    double xa[kMaxNuc][3];       // nucleus positions
    double wgt[kMaxNuc];         // z_a (2/pi^2) / P^3
};

template <typename T, int NK>
__device__ __forceinline__ void load_k1(const T* __restrict__ p, double (&v)[NK])
{
    if constexpr (sizeof(T) == 4) {
        static_assert(NK % 4 == 0, "float4 rows");
        const float4* q = reinterpret_cast<const float4*>(p);
        fft::sfor<0, NK / 4>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const float4 t = q[i];
            v[4 * i] = t.x;
            v[4 * i + 1] = t.y;
            v[4 * i + 2] = t.z;
            v[4 * i + 3] = t.w;
        });
    } else {
        const double2* q = reinterpret_cast<const double2*>(p);
        fft::sfor<0, NK / 2>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const double2 t = q[i];
            v[2 * i] = t.x;
            v[2 * i + 1] = t.y;
        });
    }
}

template <typename T, int NK>
__device__ __forceinline__ void store_k1(T* __restrict__ p, const double (&v)[NK])
{
    if constexpr (sizeof(T) == 4) {
        float4* q = reinterpret_cast<float4*>(p);
        fft::sfor<0, NK / 4>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            q[i] = make_float4((float)v[4 * i], (float)v[4 * i + 1], (float)v[4 * i + 2], (float)v[4 * i + 3]);
        });
    } else {
        double2* q = reinterpret_cast<double2*>(p);
        fft::sfor<0, NK / 2>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            q[i] = make_double2(v[2 * i], v[2 * i + 1]);
        });
    }
}

template <int NK, int R>
struct ThetaShape {
    static constexpr int P = 2 * NK;
    static constexpr int C = P / R;          // xi1 values per chunk
    static constexpr int RS = NK + 1;        // padded row length (complex)
    static constexpr int W1N = C * NK * RS;     // W1 and its odd-half twin W1o
    static constexpr int W2N = C * P * RS;
    static_assert(P % R == 0, "chunks");
    static_assert(C <= NK ? NK % C == 0 : C == 2 * NK, "chunk length");
};

// SPLIT: stages B and D as two half-transform work items per line (else one item per
// line; measured 3 % slower at N_k = 16).
template <typename T, int NK, int R, int NT, int WPE = 1, bool SPLIT = true>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_theta(T* __restrict__ fx, const double* __restrict__ kt, const ThetaArgs a,
                                             long long total)
{
    using namespace fft;
    using S = ThetaShape<NK, R>;
    constexpr int P = S::P, C = S::C, RS = S::RS;
    constexpr int LA = NK * NK, LB = C * NK, LC = C * P;
    // k1 lines owned by a thread in stages A and E (the only state kept across chunks
    // is the real result of each owned line; the input line is re-read from memory)
    constexpr int LPT = LA >= NT ? LA / NT : 1;
    static_assert(LA < NT || LA % NT == 0, "whole k1 lines per thread");
    __shared__ cd W1[S::W1N];
    __shared__ cd W1o[SPLIT ? S::W1N : 1];
    __shared__ cd W2[S::W2N];
    __shared__ cd E[3][NK];

    const int tid = threadIdx.x;

    for (long long xp = blockIdx.x; xp < total; xp += gridDim.x) {
        const long long loc = xp % a.npts;
        const int i1 = (int)(loc % a.nx[0]);
        const int i2 = (int)((loc / a.nx[0]) % a.nx[1]);
        const int i3 = (int)(loc / ((long long)a.nx[0] * a.nx[1]));
        const double xc[3] = {a.x_lo[0] + i1 * a.hx[0], a.x_lo[1] + i2 * a.hx[1], a.x_lo[2] + i3 * a.hx[2]};
        T* base = fx + xp * (long long)(NK * NK * NK);

        double th[LPT][NK];
        sfor<0, LPT>([&](auto lc) {
            sfor<0, NK>([&](auto jc) { th[decltype(lc)::value][decltype(jc)::value] = 0.0; });
        });

        for (int nu = 0; nu < a.nnuc; ++nu) {
            __syncthreads();   // E of the previous pass is no longer read
            if (tid < 3 * NK) {
                const int d = tid / NK, k = tid % NK;
                const double ph = 2.0 * (xc[d] - a.xa[nu][d]) * a.hk[d] * k;
                double s, c;
                sincos(ph, &s, &c);
                E[d][k] = cd{c, -s};                                  // e^{-i phi_d k}
            }
            __syncthreads();
            const double w = a.wgt[nu];
            sfor<0, R>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                // ---- A: k1 forward of this chunk (xi1 = r + R m) from the modulated line
                sfor<0, LPT>([&](auto lc) {
                    const int la = tid + decltype(lc)::value * NT;
                    if (la < LA) {
                        const int k2 = la % NK, k3 = la / NK;
                        double fv[NK];
                        load_k1<T, NK>(base + (long long)la * NK, fv);
                        const cd e23 = cmul(E[1][k2], E[2][k3]);
                        cd z[NK];
                        sfor<0, NK>([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            const cd e = cmul(E[0][j], e23);
                            z[j] = cd{e.re * fv[j], e.im * fv[j]};
                        });
                        cd Y[C];
                        if constexpr (C <= NK) {
                            sfor<0, C>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                cd s{0.0, 0.0};
                                sfor<0, NK / C>([&](auto sc) {
                                    constexpr int k = j + decltype(sc)::value * C;
                                    s = cadd(s, tmul<(long long)r * k, P, -1>(z[k]));
                                });
                                Y[j] = s;
                            });
                            transform<C, -1>(Y);
                        } else {
                            cd y[NK];
                            sfor<0, NK>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                y[j] = tmul<(long long)r * j, P, -1>(z[j]);
                            });
                            fft_fwd_padded<NK>(y, Y);
                        }
                        sfor<0, C>([&](auto mc) {
                            constexpr int m = decltype(mc)::value;
                            W1[(m * NK + k3) * RS + k2] = Y[m];
                        });
                    }
                });
                __syncthreads();
                // ---- B: k2 forward, zero-padded to P.  The two halves of a line (even
                // and odd outputs: transforms of x_j and of x_j w^j) go to two work items,
                // so 2 LB items keep every thread busy; h is uniform across a wave.
                if constexpr (SPLIT) {
                    for (int it = tid; it < 2 * LB; it += NT) {
                        const int h = it / LB, ln = it % LB;
                        const int m = ln / NK, q3 = ln % NK;
                        cd row[NK];
                        sfor<0, NK>([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            const cd x = W1[(m * NK + q3) * RS + j];
                            row[j] = h ? tmul<j, P, -1>(x) : x;
                        });
                        transform<NK, -1>(row);
                        sfor<0, NK>([&](auto fc) {
                            constexpr int f = decltype(fc)::value;
                            W2[(m * P + 2 * f + h) * RS + q3] = row[f];
                        });
                    }
                } else {
                    for (int ln = tid; ln < LB; ln += NT) {
                        const int m = ln / NK, q3 = ln % NK;
                        cd row[NK], Y[P];
                        sfor<0, NK>([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            row[j] = W1[(m * NK + q3) * RS + j];
                        });
                        fft_fwd_padded<NK>(row, Y);
                        sfor<0, P>([&](auto fc) {
                            constexpr int f = decltype(fc)::value;
                            W2[(m * P + f) * RS + q3] = Y[f];
                        });
                    }
                }
                __syncthreads();
                // ---- C: the k3 convolution of every (xi1, xi2) line, in place: the first NK
                // outputs of the period-P circular convolution of the zero-padded line are
                // a Toeplitz product with the kernel transformed along k1 and k2 only,
                // o_j = sum_j' row_j' K(|j - j'|), K real (see kt below)
                for (int ln = tid; ln < LC; ln += NT) {
                    const int m = ln / P, f2 = ln % P;
                    cd row[NK], o[NK];
                    double kk[NK];
                    const double2* kr = reinterpret_cast<const double2*>(kt + ((long long)(r + R * m) * P + f2) * NK);
                    sfor<0, NK / 2>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        const double2 t = kr[q];
                        kk[2 * q] = t.x;
                        kk[2 * q + 1] = t.y;
                    });
                    sfor<0, NK>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        row[j] = W2[(m * P + f2) * RS + j];
                    });
                    sfor<0, NK>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        double re = 0.0, im = 0.0;
                        sfor<0, NK>([&](auto ic) {
                            constexpr int i = decltype(ic)::value;
                            constexpr int d = j > i ? j - i : i - j;
                            re = fma(kk[d], row[i].re, re);
                            im = fma(kk[d], row[i].im, im);
                        });
                        o[j] = cd{re, im};
                    });
                    sfor<0, NK>([&](auto jc) {
                        constexpr int j = decltype(jc)::value;
                        W2[(m * P + f2) * RS + j] = o[j];
                    });
                }
                __syncthreads();
                // ---- D: k2 inverse, first NK outputs, as two halves: the inverse of the
                // even inputs into W1, the inverse of the odd inputs times w^-j into W1o
                // (stage E adds them)
                if constexpr (SPLIT) {
                    for (int it = tid; it < 2 * LB; it += NT) {
                        const int h = it / LB, ln = it % LB;
                        const int m = ln / NK, q3 = ln % NK;
                        cd col[NK];
                        sfor<0, NK>([&](auto fc) {
                            constexpr int f = decltype(fc)::value;
                            col[f] = W2[(m * P + 2 * f + h) * RS + q3];
                        });
                        transform<NK, +1>(col);
                        cd* dst = h ? W1o : W1;
                        sfor<0, NK>([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            dst[(m * NK + q3) * RS + j] = h ? tmul<j, P, +1>(col[j]) : col[j];
                        });
                    }
                } else {
                    for (int ln = tid; ln < LB; ln += NT) {
                        const int m = ln / NK, q3 = ln % NK;
                        cd col[P], o[NK];
                        sfor<0, P>([&](auto fc) {
                            constexpr int f = decltype(fc)::value;
                            col[f] = W2[(m * P + f) * RS + q3];
                        });
                        fft_inv_half<NK>(col, o);
                        sfor<0, NK>([&](auto jc) {
                            constexpr int j = decltype(jc)::value;
                            W1[(m * NK + q3) * RS + j] = o[j];
                        });
                    }
                }
                __syncthreads();
                // ---- E: k1 inverse of this chunk, demodulated, into the real result
                sfor<0, LPT>([&](auto lc) {
                    constexpr int l = decltype(lc)::value;
                    const int la = tid + l * NT;
                    if (la < LA) {
                        const int k2 = la % NK, k3 = la / NK;
                        const cd e23c = conj(cmul(E[1][k2], E[2][k3]));
                        cd v[C];
                        sfor<0, C>([&](auto mc) {
                            constexpr int m = decltype(mc)::value;
                            v[m] = SPLIT ? cadd(W1[(m * NK + k3) * RS + k2], W1o[(m * NK + k3) * RS + k2])
                                         : W1[(m * NK + k3) * RS + k2];
                        });
                        auto put = [&](auto kc, cd x) {
                            constexpr int k = decltype(kc)::value;
                            const cd d = cmul(conj(E[0][k]), e23c);             // e^{+i phi.p}
                            const cd t = cmul(d, tmul<(long long)r * k, P, +1>(x));
                            th[l][k] += w * t.im;
                        };
                        if constexpr (C <= NK) {
                            transform<C, +1>(v);
                            sfor<0, NK>([&](auto kc) { put(kc, v[decltype(kc)::value % C]); });
                        } else {
                            cd vh[NK];
                            fft_inv_half<NK>(v, vh);
                            sfor<0, NK>([&](auto kc) { put(kc, vh[decltype(kc)::value]); });
                        }
                    }
                });
                __syncthreads();
            });
        }
        __syncthreads();   // every line of this x-point is read (stage A) before any is written
        sfor<0, LPT>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            const int la = tid + l * NT;
            if (la < LA) store_k1<T, NK>(base + (long long)la * NK, th[l]);
        });
    }
}

// out[b][c][r] = in[b][r][c] for an (rows x cols) matrix per batch member; 64 x 64
// tiles through LDS, 256 threads, coalesced on both sides.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ in, T* __restrict__ out, long long rows,
                                                  long long cols)
{
    __shared__ T tile[64][65];
    const long long b = blockIdx.z;
    const long long r0 = (long long)blockIdx.y * 64, c0 = (long long)blockIdx.x * 64;
    const T* src = in + b * rows * cols;
    T* dst = out + b * rows * cols;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const long long r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) tile[i][tx] = src[r * cols + c];
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const long long c = c0 + i, r = r0 + tx;
        if (r < rows && c < cols) dst[c * rows + r] = tile[tx][i];
    }
}

}  // namespace chasm

// chasm_fft.hpp -- small complex FP64 transforms held in registers, with compile-time
// twiddles, for the truncated-kernel evaluation of Theta_V (Sec. 4).
//
// Conventions: forward X[f] = sum_j x[j] e^{-2 pi i j f / L}; inverse without the
// 1/L factor, x[j] = sum_f X[f] e^{+2 pi i j f / L}.  L is a power of two.  Arrays are
// register arrays indexed only by compile-time constants, so every permutation is a
// renaming and every twiddle an immediate.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace chasm {
namespace fft {

struct cd {
    double re, im;
};

__host__ __device__ __forceinline__ constexpr cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ __forceinline__ constexpr cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ __forceinline__ cd cmul(cd a, cd b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ __forceinline__ constexpr cd conj(cd a) { return {a.re, -a.im}; }

template <int B, int E, typename F>
__host__ __device__ __forceinline__ constexpr void sfor(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// ---- constexpr sine / cosine (Taylor series on |r| <= pi/4 after quadrant reduction)
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double r)
{
    double term = r, sum = r;
    for (int n = 1; n < 14; ++n) {
        term *= -r * r / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}

constexpr double taylor_cos(double r)
{
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 14; ++n) {
        term *= -r * r / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}

// e^{sign 2 pi i k / L}, reduced on the integers first: k/L in eighths of a turn.
constexpr cd twiddle(long long k, long long L, int sign)
{
    k %= L;
    if (k < 0) k += L;
    // quadrant q = round(4k/L), remainder angle r = 2 pi (k/L - q/4) in [-pi/4, pi/4]
    const long long q = (8 * k + L) / (2 * L);
    const double frac = (double)(4 * k - q * L) / (double)(4 * L);   // in [-1/8, 1/8]
    const double r = 2.0 * kPi * frac;
    const double c = taylor_cos(r), s = taylor_sin(r);
    double re = 0, im = 0;
    switch ((int)(q % 4)) {
        case 0: re = c; im = s; break;
        case 1: re = -s; im = c; break;
        case 2: re = -c; im = -s; break;
        default: re = s; im = -c; break;
    }
    return {re, sign * im};
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

constexpr int bitrev(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

// Multiply by the compile-time twiddle e^{sign 2 pi i k / L}; the exact cases cost no
// multiplication.
template <long long K, long long L, int SIGN>
__host__ __device__ __forceinline__ cd tmul(cd a)
{
    constexpr long long k = ((K % L) + L) % L;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (4 * k == L) {   // e^{sign i pi/2} = sign i
        return SIGN > 0 ? cd{-a.im, a.re} : cd{a.im, -a.re};
    } else if constexpr (2 * k == L) {
        return {-a.re, -a.im};
    } else if constexpr (4 * k == 3 * L) {
        return SIGN > 0 ? cd{a.im, -a.re} : cd{-a.im, a.re};
    } else {
        constexpr cd w = twiddle(k, L, SIGN);
        return cmul(a, w);
    }
}

// In-place radix-2 transform of length L (SIGN -1 forward, +1 inverse), natural order
// in and out.
template <int L, int SIGN>
__host__ __device__ __forceinline__ void transform(cd (&v)[L])
{
    constexpr int bits = ilog2(L);
    static_assert((1 << bits) == L, "power of two");
    sfor<0, L>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int j = bitrev(i, bits);
        if constexpr (i < j) {
            const cd t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    });
    sfor<0, bits>([&](auto sc) {
        constexpr int half = 1 << decltype(sc)::value;
        constexpr int len = 2 * half;
        sfor<0, L / len>([&](auto bc) {
            constexpr int base = decltype(bc)::value * len;
            sfor<0, half>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const cd a = v[base + j];
                const cd b = tmul<j, len, SIGN>(v[base + j + half]);
                v[base + j] = cadd(a, b);
                v[base + j + half] = csub(a, b);
            });
        });
    });
}

// Forward transform of length 2H whose inputs H..2H-1 are zero: from the H given
// values, out[0..2H) (even outputs = transform of x, odd = transform of x_j w^j).
template <int H>
__host__ __device__ __forceinline__ void fft_fwd_padded(const cd (&x)[H], cd (&out)[2 * H])
{
    cd e[H], o[H];
    sfor<0, H>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        e[j] = x[j];
        o[j] = tmul<j, 2 * H, -1>(x[j]);
    });
    transform<H, -1>(e);
    transform<H, -1>(o);
    sfor<0, H>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        out[2 * m] = e[m];
        out[2 * m + 1] = o[m];
    });
}

// Inverse transform of length 2H keeping only outputs 0..H-1.
template <int H>
__host__ __device__ __forceinline__ void fft_inv_half(const cd (&X)[2 * H], cd (&out)[H])
{
    cd e[H], o[H];
    sfor<0, H>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        e[m] = X[2 * m];
        o[m] = X[2 * m + 1];
    });
    transform<H, +1>(e);
    transform<H, +1>(o);
    sfor<0, H>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        out[j] = cadd(e[j], tmul<j, 2 * H, +1>(o[j]));
    });
}

}  // namespace fft
}  // namespace chasm

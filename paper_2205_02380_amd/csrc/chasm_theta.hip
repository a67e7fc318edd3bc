// chasm_theta.hip -- C ABI of the truncated-kernel evaluation of Theta_V (Sec. 4):
// descriptor validation, the FP64 tensor T of eq. 4.9 and its transform on the host,
// kernel selection, and the apply sequence (transpose to x-major, per-x-point FFT
// convolution, transpose back).  See include/chasm_theta.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/chasm_theta.h"
#include "chasm_theta.hpp"
#include "chasm_theta_big.hpp"

namespace chasm {

void set_last_error(const std::string& msg);

// ---------------------------------------------------------------------------
// Sine integral Si(x) = int_0^x sin(t)/t dt.  |x| <= 4: the Maclaurin series
// sum_n (-1)^n x^{2n+1} / ((2n+1) (2n+1)!).  Beyond: Si(x) = pi/2 + Im E1(i x)
// (E1(i x) = -Ci(x) + i (Si(x) - pi/2)), with E1 from its continued fraction
// e^{z} E1(z) = 1/(z+1 - 1/(z+3 - 4/(z+5 - 9/(z+7 - ...)))) evaluated by the modified
// Lentz method.
static double sine_integral(double x)
{
    const double ax = std::fabs(x);
    double r;
    if (ax <= 4.0) {
        double p = ax, sum = ax;
        for (int n = 1; n < 60; ++n) {
            p *= -ax * ax / ((2.0 * n) * (2.0 * n + 1.0));
            const double t = p / (2.0 * n + 1.0);
            sum += t;
            if (std::fabs(t) < 1e-18 * std::fabs(sum)) break;
        }
        r = sum;
    } else {
        const std::complex<double> z(0.0, ax);
        const double tiny = 1e-300;
        std::complex<double> b = z + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
        for (int i = 1; i < 10000; ++i) {
            const double an = -(double)i * (double)i;
            b += 2.0;
            d = 1.0 / (an * d + b);
            c = b + an / c;
            const std::complex<double> del = c * d;
            h *= del;
            if (std::abs(del - 1.0) < 1e-16) break;
        }
        r = M_PI / 2 + (h * std::exp(-z)).imag();
    }
    return x < 0 ? -r : r;
}

// Fourier transform of |k|^-2 truncated at |k| <= D, at |xi| = q (Sec. 4.1).
static double uhat_truncated(double q, double D)
{
    return q > 0 ? 4.0 * M_PI * sine_integral(q * D) / q : 4.0 * M_PI * D;
}

// cos(2 pi a / m) with a reduced modulo m first.
static double cos_turn(long long a, long long m)
{
    a %= m;
    if (a < 0) a += m;
    return std::cos(2.0 * M_PI * (double)a / (double)m);
}

// T_p of eq. 4.9 for p_d in [0, nk_d): the real sum (1/M^3) sum_n Uhat_D(xi_n)
// prod_d cos(2 pi p_d n_d / M_d) over the dual set n_d in [-M_d/2, M_d/2), M_d = 3 nk_d,
// xi_{n,d} = 2 pi n_d / (M_d hk_d) (eq. 4.10), in three separable passes.  The odd
// parts cancel between n_d and -n_d, and the unpaired n_d = -M_d/2 has a zero sine.
// Output [p3][p2][p1]; T is even in every p_d.
static void tensor_positive(const int nk[3], const double hk[3], std::vector<double>& T)
{
    const int M[3] = {3 * nk[0], 3 * nk[1], 3 * nk[2]};
    double D2 = 0.0;
    for (int d = 0; d < 3; ++d) D2 += (nk[d] * hk[d]) * (nk[d] * hk[d]);
    const double D = std::sqrt(D2);
    std::vector<double> xi[3];
    for (int d = 0; d < 3; ++d) {
        xi[d].resize(M[d]);
        for (int i = 0; i < M[d]; ++i) xi[d][i] = 2.0 * M_PI * (i - M[d] / 2) / (M[d] * hk[d]);
    }
    std::vector<double> cs[3];   // cs[d][p * M + i] = cos(2 pi p n_i / M)
    for (int d = 0; d < 3; ++d) {
        cs[d].resize((size_t)nk[d] * M[d]);
        for (int p = 0; p < nk[d]; ++p)
            for (int i = 0; i < M[d]; ++i) cs[d][(size_t)p * M[d] + i] = cos_turn((long long)p * (i - M[d] / 2), M[d]);
    }
    // pass 1 over n1: A1[n3][n2][p1]
    std::vector<double> A1((size_t)M[2] * M[1] * nk[0]);
    std::vector<double> U(M[0]);
    for (int i3 = 0; i3 < M[2]; ++i3)
        for (int i2 = 0; i2 < M[1]; ++i2) {
            for (int i1 = 0; i1 < M[0]; ++i1)
                U[i1] = uhat_truncated(std::sqrt(xi[0][i1] * xi[0][i1] + xi[1][i2] * xi[1][i2] + xi[2][i3] * xi[2][i3]), D);
            for (int p1 = 0; p1 < nk[0]; ++p1) {
                double s = 0.0;
                for (int i1 = 0; i1 < M[0]; ++i1) s += U[i1] * cs[0][(size_t)p1 * M[0] + i1];
                A1[((size_t)i3 * M[1] + i2) * nk[0] + p1] = s;
            }
        }
    // pass 2 over n2: A2[n3][p2][p1]
    std::vector<double> A2((size_t)M[2] * nk[1] * nk[0]);
    for (int i3 = 0; i3 < M[2]; ++i3)
        for (int p2 = 0; p2 < nk[1]; ++p2)
            for (int p1 = 0; p1 < nk[0]; ++p1) {
                double s = 0.0;
                for (int i2 = 0; i2 < M[1]; ++i2)
                    s += A1[((size_t)i3 * M[1] + i2) * nk[0] + p1] * cs[1][(size_t)p2 * M[1] + i2];
                A2[((size_t)i3 * nk[1] + p2) * nk[0] + p1] = s;
            }
    // pass 3 over n3, with the 1/M^3 of the inverse DFT
    const double scale = 1.0 / ((double)M[0] * M[1] * M[2]);
    T.assign((size_t)nk[2] * nk[1] * nk[0], 0.0);
    for (int p3 = 0; p3 < nk[2]; ++p3)
        for (int p2 = 0; p2 < nk[1]; ++p2)
            for (int p1 = 0; p1 < nk[0]; ++p1) {
                double s = 0.0;
                for (int i3 = 0; i3 < M[2]; ++i3)
                    s += A2[((size_t)i3 * nk[1] + p2) * nk[0] + p1] * cs[2][(size_t)p3 * M[2] + i3];
                T[((size_t)p3 * nk[1] + p2) * nk[0] + p1] = s * scale;
            }
}

// T placed circularly with period P_d = 2 nk_d (entries at |q_d| = nk_d are zero),
// transformed along k1 and k2 only: B(xi1, xi2, q3) = sum_{q1, q2} T_q cos(2 pi (q1 xi1 /
// P1 + q2 xi2 / P2)), real since T is even in each coordinate.  The full transform would
// be That(xi) = sum_{|q3| < nk3} B(xi1, xi2, |q3|) e^{2 pi i q3 xi3 / P3}, so transforming
// a zero-padded k3 line, multiplying by That and transforming back (without 1/P3) gives,
// at the first nk3 outputs, o_j = sum_j' P3 B(xi1, xi2, |j - j'|) row_j'.  Output
// kt[xi1][xi2][q3] = P3 B(xi1, xi2, q3), q3 < nk3 (q3 fastest), the order the kernel
// reads it in.
static void tensor_partial(const int nk[3], const std::vector<double>& T, std::vector<double>& kt)
{
    const int P[3] = {2 * nk[0], 2 * nk[1], 2 * nk[2]};
    // per axis: g(xi) = g(0) + 2 sum_{q=1}^{nk-1} g(q) cos(2 pi q xi / P)
    auto wcos = [&](int d, int q, int f) { return (q == 0 ? 1.0 : 2.0) * cos_turn((long long)q * f, P[d]); };
    std::vector<double> B1((size_t)nk[2] * nk[1] * P[0]);   // [q3][q2][xi1]
    for (int q3 = 0; q3 < nk[2]; ++q3)
        for (int q2 = 0; q2 < nk[1]; ++q2)
            for (int f1 = 0; f1 < P[0]; ++f1) {
                double s = 0.0;
                for (int q1 = 0; q1 < nk[0]; ++q1) s += T[((size_t)q3 * nk[1] + q2) * nk[0] + q1] * wcos(0, q1, f1);
                B1[((size_t)q3 * nk[1] + q2) * P[0] + f1] = s;
            }
    kt.assign((size_t)P[0] * P[1] * nk[2], 0.0);
    for (int q3 = 0; q3 < nk[2]; ++q3)
        for (int f2 = 0; f2 < P[1]; ++f2)
            for (int f1 = 0; f1 < P[0]; ++f1) {
                double s = 0.0;
                for (int q2 = 0; q2 < nk[1]; ++q2) s += B1[((size_t)q3 * nk[1] + q2) * P[0] + f1] * wcos(1, q2, f2);
                kt[((size_t)f1 * P[1] + f2) * nk[2] + q3] = P[2] * s;
            }
}

// ---------------------------------------------------------------------------
// Compiled kernels: (storage type, nk) -> chunk count R and block size of the one-block
// form (nk 8, 16), and the staged form over batches of x-points (nk 16, 32, 64).
using BigFn = hipError_t (*)(void* fx, const double* kt, const ThetaArgs& a, fft::cd* W, double* acc,
                             long long total, long long X, hipStream_t s);

struct ThetaKernels {
    int dtype, nk;
    hipError_t (*theta)(void* fx, const double* kt, const ThetaArgs& a, long long total, hipStream_t s);
    hipError_t (*transpose)(const void* in, void* out, long long rows, long long cols, int batch, hipStream_t s);
    BigFn big;                 // staged form (nullptr: none)
};

template <typename K>
static long long resident(K k, int threads)
{
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, threads, 0) != hipSuccess) return 0;
    return (long long)ncu * (per > 0 ? per : 1);
}

template <typename T, int NK, int R, int NT>
static hipError_t launch_theta(void* fx, const double* kt, const ThetaArgs& a, long long total, hipStream_t s)
{
    auto k = k_theta<T, NK, R, NT>;
    const long long res = resident(k, NT);
    const unsigned grid = (unsigned)(res > 0 && res < total ? res : total);
    hipLaunchKernelGGL(k, dim3(grid), dim3(NT), 0, s, static_cast<T*>(fx), kt, a, total);
    return hipGetLastError();
}

// Staged form: x-points in batches of X; per batch and nucleus the three stages.
template <typename T, int NK>
static hipError_t launch_big(void* fx, const double* kt, const ThetaArgs& a, fft::cd* W, double* acc,
                             long long total, long long X, hipStream_t s)
{
    using B = BigShape<NK>;
    for (long long x0 = 0; x0 < total; x0 += X) {
        const long long nb = total - x0 < X ? total - x0 : X;
        for (int nu = 0; nu < a.nnuc; ++nu) {
            hipLaunchKernelGGL((k_thA<T, NK>), dim3((unsigned)(nb * B::BPX)), dim3(64), 0, s,
                               static_cast<const T*>(fx), W, a, x0, nu);
            hipLaunchKernelGGL((k_thBCD<NK>), dim3((unsigned)(nb * B::P)), dim3(B::NTB), 0, s, W, kt);
            hipLaunchKernelGGL((k_thE<T, NK>), dim3((unsigned)(nb * B::BPX)), dim3(64), 0, s, W, acc,
                               static_cast<T*>(fx), a, x0, nu, nu == 0 ? 1 : 0, nu == a.nnuc - 1 ? 1 : 0);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <typename T>
static hipError_t launch_transpose(const void* in, void* out, long long rows, long long cols, int batch, hipStream_t s)
{
    const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64), (unsigned)batch);
    hipLaunchKernelGGL(k_transpose<T>, grid, dim3(256), 0, s, static_cast<const T*>(in), static_cast<T*>(out), rows,
                       cols);
    return hipGetLastError();
}

static const ThetaKernels kThetaKernels[] = {
    {CHASM_F32, 8, launch_theta<float, 8, 1, 256>, launch_transpose<float>, nullptr},
    {CHASM_F64, 8, launch_theta<double, 8, 1, 256>, launch_transpose<double>, nullptr},
    {CHASM_F32, 16, launch_theta<float, 16, 4, 256>, launch_transpose<float>, launch_big<float, 16>},
    {CHASM_F64, 16, launch_theta<double, 16, 4, 256>, launch_transpose<double>, launch_big<double, 16>},
    {CHASM_F32, 32, nullptr, launch_transpose<float>, launch_big<float, 32>},
    {CHASM_F64, 32, nullptr, launch_transpose<double>, launch_big<double, 32>},
    {CHASM_F32, 64, nullptr, launch_transpose<float>, launch_big<float, 64>},
    {CHASM_F64, 64, nullptr, launch_transpose<double>, launch_big<double, 64>},
};

static const ThetaKernels* find_theta(int dtype, int nk)
{
    for (const ThetaKernels& k : kThetaKernels)
        if (k.dtype == dtype && k.nk == nk) return &k;
    return nullptr;
}

// Staged form: x-points per batch (intermediate W of X * 2 nk^3 complex values, at most
// about 2 GiB) and whether a handle uses it.
static long long big_batch(int nk, long long total)
{
    const long long per = 2LL * nk * nk * nk * 16;
    long long X = (2LL << 30) / per;
    if (X < 1) X = 1;
    return X < total ? X : total;
}

static bool use_big(const chasm_theta_desc* d, const ThetaKernels* ks)
{
    return !ks->theta || (d->flags & CHASM_THETA_FLAG_STAGED);
}

}  // namespace chasm

using namespace chasm;

struct chasm_theta_s {
    chasm_theta_desc desc;
    hipStream_t stream = nullptr;
    const ThetaKernels* ks = nullptr;
    double* kt = nullptr;               // kernel transformed along k1, k2 (tensor_partial)
    void* ws = nullptr;
    bool big = false;                   // staged form
    long long X = 0;                    // x-points per batch of the staged form
    fft::cd* W = nullptr;               // its complex intermediate
    double* acc = nullptr;              // its sum over nuclei (more than one nucleus)
    ThetaArgs args{};
    long long npts = 0, nkp = 0;
    bool poisoned = false;
};

static chasm_status tfail(chasm_status st, const std::string& msg)
{
    set_last_error(msg);
    return st;
}

static chasm_status validate(const chasm_theta_desc* d, const ThetaKernels** ks)
{
    if (!d) return tfail(CHASM_EINVAL, "descriptor is NULL");
    for (int a = 0; a < 3; ++a) {
        if (d->nx[a] < 1 || d->nk[a] < 2) return tfail(CHASM_EINVAL, "nx must be >= 1 and nk >= 2 on every axis");
        if (!(d->x_hi[a] > d->x_lo[a]) || !(d->k_hi[a] > d->k_lo[a]) || !std::isfinite(d->x_lo[a]) ||
            !std::isfinite(d->x_hi[a]) || !std::isfinite(d->k_lo[a]) || !std::isfinite(d->k_hi[a]))
            return tfail(CHASM_EINVAL, "every axis needs finite bounds with hi > lo");
        if (d->nk[a] % 2) return tfail(CHASM_EINVAL, "nk must be even (the dual index set of eq. 4.10)");
    }
    if (d->nnuc < 1 || d->nnuc > CHASM_THETA_MAX_NUCLEI) return tfail(CHASM_EINVAL, "nnuc must be in 1..4");
    for (int i = 0; i < d->nnuc; ++i) {
        if (!std::isfinite(d->z_nuc[i])) return tfail(CHASM_EINVAL, "nucleus charge is not finite");
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(d->x_nuc[i][a])) return tfail(CHASM_EINVAL, "nucleus position is not finite");
    }
    if (d->dtype != CHASM_F32 && d->dtype != CHASM_F64) return tfail(CHASM_EINVAL, "dtype must be CHASM_F32 or CHASM_F64");
    if (d->nbatch < 1) return tfail(CHASM_EINVAL, "nbatch must be >= 1");
    const long long pts = (long long)d->nx[0] * d->nx[1] * d->nx[2] * d->nk[0] * d->nk[1] * d->nk[2];
    if (pts <= 0 || pts > (1LL << 40) / d->nbatch) return tfail(CHASM_EINVAL, "grid too large");
    if (d->flags & ~(uint32_t)CHASM_THETA_FLAG_STAGED) return tfail(CHASM_EINVAL, "unknown flags");
    if (d->nk[0] != d->nk[1] || d->nk[1] != d->nk[2])
        return tfail(CHASM_EUNSUPPORTED, "kernels are built for equal nk on the three axes");
    const ThetaKernels* k = find_theta(d->dtype, d->nk[0]);
    if (!k) return tfail(CHASM_EUNSUPPORTED, "no kernel for this nk (built: 8, 16, 32, 64)");
    if ((d->flags & CHASM_THETA_FLAG_STAGED) && !k->big)
        return tfail(CHASM_EUNSUPPORTED, "the staged form is built for nk 16, 32, 64");
    if (ks) *ks = k;
    return CHASM_OK;
}

static void desc_hk(const chasm_theta_desc* d, int nk[3], double hk[3])
{
    for (int a = 0; a < 3; ++a) {
        nk[a] = d->nk[a];
        hk[a] = (d->k_hi[a] - d->k_lo[a]) / d->nk[a];
    }
}

extern "C" {

chasm_status chasm_theta_workspace_bytes(const chasm_theta_desc* desc, size_t* bytes)
{
    const ThetaKernels* ks = nullptr;
    chasm_status st = validate(desc, &ks);
    if (st != CHASM_OK) return st;
    if (!bytes) return tfail(CHASM_EINVAL, "bytes is NULL");
    const size_t es = desc->dtype == CHASM_F64 ? 8 : 4;
    const size_t pts = (size_t)desc->nx[0] * desc->nx[1] * desc->nx[2] * desc->nk[0] * desc->nk[1] * desc->nk[2];
    const size_t P3 = (size_t)8 * desc->nk[0] * desc->nk[1] * desc->nk[2];
    *bytes = pts * desc->nbatch * es + P3 * sizeof(double) + 512;
    if (use_big(desc, ks)) {
        const long long nk = desc->nk[0];
        const long long X = big_batch((int)nk, (long long)desc->nx[0] * desc->nx[1] * desc->nx[2] * desc->nbatch);
        *bytes += (size_t)X * 2 * nk * nk * nk * 16 + 256;
        if (desc->nnuc > 1) *bytes += (size_t)X * nk * nk * nk * 8 + 256;
    }
    return CHASM_OK;
}

chasm_status chasm_theta_tensor(const chasm_theta_desc* desc, double* t_host)
{
    chasm_status st = validate(desc, nullptr);
    if (st != CHASM_OK && st != CHASM_EUNSUPPORTED) return st;
    if (!t_host) return tfail(CHASM_EINVAL, "t_host is NULL");
    int nk[3];
    double hk[3];
    desc_hk(desc, nk, hk);
    std::vector<double> T;
    tensor_positive(nk, hk, T);
    const int w1 = 2 * nk[0] - 1, w2 = 2 * nk[1] - 1, w3 = 2 * nk[2] - 1;
    for (int q3 = 0; q3 < w3; ++q3)
        for (int q2 = 0; q2 < w2; ++q2)
            for (int q1 = 0; q1 < w1; ++q1) {
                const int p3 = std::abs(q3 - (nk[2] - 1)), p2 = std::abs(q2 - (nk[1] - 1)), p1 = std::abs(q1 - (nk[0] - 1));
                t_host[((size_t)q3 * w2 + q2) * w1 + q1] = T[((size_t)p3 * nk[1] + p2) * nk[0] + p1];
            }
    return CHASM_OK;
}

chasm_status chasm_theta_create(const chasm_theta_desc* desc, void* hip_stream, chasm_theta_t* out)
{
    if (!out) return tfail(CHASM_EINVAL, "out is NULL");
    *out = nullptr;
    const ThetaKernels* ks = nullptr;
    chasm_status st = validate(desc, &ks);
    if (st != CHASM_OK) return st;

    int nk[3];
    double hk[3];
    desc_hk(desc, nk, hk);
    std::vector<double> T, KT;
    tensor_positive(nk, hk, T);
    tensor_partial(nk, T, KT);

    chasm_theta_s* h = new (std::nothrow) chasm_theta_s();
    if (!h) return tfail(CHASM_ENOMEM, "host allocation failed");
    h->desc = *desc;
    h->stream = (hipStream_t)hip_stream;
    h->ks = ks;
    h->npts = (long long)desc->nx[0] * desc->nx[1] * desc->nx[2];
    h->nkp = (long long)nk[0] * nk[1] * nk[2];
    auto bail = [&](chasm_status s, const std::string& m) {
        chasm_theta_destroy(h);
        return tfail(s, m);
    };
    if (hipMalloc((void**)&h->kt, KT.size() * sizeof(double)) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(symbol) failed");
    if (hipMemcpyAsync(h->kt, KT.data(), KT.size() * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
        hipSuccess)
        return bail(CHASM_EDEVICE, "symbol upload failed");
    const size_t es = desc->dtype == CHASM_F64 ? 8 : 4;
    if (hipMalloc(&h->ws, (size_t)h->npts * h->nkp * desc->nbatch * es) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(workspace) failed");
    h->big = use_big(desc, ks);
    if (h->big) {
        const long long nkk = nk[0];
        h->X = big_batch(nk[0], h->npts * desc->nbatch);
        if (hipMalloc((void**)&h->W, (size_t)h->X * 2 * nkk * nkk * nkk * sizeof(fft::cd)) != hipSuccess)
            return bail(CHASM_ENOMEM, "hipMalloc(staged intermediate) failed");
        if (desc->nnuc > 1 && hipMalloc((void**)&h->acc, (size_t)h->X * nkk * nkk * nkk * sizeof(double)) != hipSuccess)
            return bail(CHASM_ENOMEM, "hipMalloc(staged accumulator) failed");
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(CHASM_EDEVICE, "stream synchronize failed");

    ThetaArgs& a = h->args;
    a.npts = h->npts;
    a.nnuc = desc->nnuc;
    const double P3 = 8.0 * nk[0] * nk[1] * nk[2];
    for (int d = 0; d < 3; ++d) {
        a.nx[d] = desc->nx[d];
        a.x_lo[d] = desc->x_lo[d];
        a.hx[d] = (desc->x_hi[d] - desc->x_lo[d]) / desc->nx[d];
        a.hk[d] = hk[d];
    }
    for (int i = 0; i < desc->nnuc; ++i) {
        for (int d = 0; d < 3; ++d) a.xa[i][d] = desc->x_nuc[i][d];
        a.wgt[i] = desc->z_nuc[i] * (2.0 / (M_PI * M_PI)) / P3;     // z_a 4/c_{3,1}, c_{3,1} = 2 pi^2; 1/P^3 of the inverse
    }
    *out = h;
    return CHASM_OK;
}

chasm_status chasm_theta_apply(chasm_theta_t h, const void* f_dev, void* out_dev)
{
    if (!h || !f_dev || !out_dev) return tfail(CHASM_EINVAL, "NULL argument");
    if (h->poisoned) return tfail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    const int nb = h->desc.nbatch;
    hipError_t e = h->ks->transpose(f_dev, h->ws, h->nkp, h->npts, nb, h->stream);
    if (e == hipSuccess)
        e = h->big ? h->ks->big(h->ws, h->kt, h->args, h->W, h->acc, h->npts * nb, h->X, h->stream)
                   : h->ks->theta(h->ws, h->kt, h->args, h->npts * nb, h->stream);
    if (e == hipSuccess) e = h->ks->transpose(h->ws, out_dev, h->npts, h->nkp, nb, h->stream);
    if (e != hipSuccess) {
        h->poisoned = true;
        return tfail(CHASM_EDEVICE, std::string("theta launch: ") + hipGetErrorString(e));
    }
    return CHASM_OK;
}

chasm_status chasm_theta_destroy(chasm_theta_t h)
{
    if (!h) return CHASM_OK;
    if (h->stream) hipStreamSynchronize(h->stream);
    if (h->kt) hipFree(h->kt);
    if (h->ws) hipFree(h->ws);
    if (h->W) hipFree(h->W);
    if (h->acc) hipFree(h->acc);
    delete h;
    return CHASM_OK;
}

}  // extern "C"

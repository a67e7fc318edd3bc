// chasm_lpc1.hip -- the LPC1 time step (Sec. 2.2) built from the characteristic step
// (chasm_advect.h) and the truncated-kernel Theta_V (chasm_theta.h).  See
// include/chasm_lpc1.h.
//
// State: the caller's field f, the library's fields G and Y.  One step:
//   G = Theta[f]                (theta apply, f -> G)
//   f = A f,  G = A G           (two advection handles on the same stream, one per field)
//   Y = f + tau G               (predictor)
//   Y = Theta[Y]                (in place)
//   f = f + tau/2 (G + Y)       (corrector)
// f is stepped in place, so no step copies the field in or out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/chasm_lpc1.h"

namespace chasm {
void set_last_error(const std::string& msg);

// mode 0: y = x0 + c x1;  mode 1: x0 = x0 + c (x1 + y).  Grid-stride loop, one element
// per lane per iteration (HBM-bound: 12 or 16 bytes per element).
template <typename T>
__global__ __launch_bounds__(256) void k_lpc1_combine(T* __restrict__ x0, const T* __restrict__ x1, T* __restrict__ y,
                                                     long long n, double c, int mode)
{
    const T cc = (T)c;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        if (mode == 0)
            y[i] = fma(cc, x1[i], x0[i]);
        else
            x0[i] = fma(cc, x1[i] + y[i], x0[i]);
    }
}

}  // namespace chasm

using namespace chasm;

struct chasm_lpc1_s {
    chasm_advect_t adv_f = nullptr;   // characteristic step of the caller's field
    chasm_advect_t adv_g = nullptr;   // characteristic step of G
    chasm_theta_t th = nullptr;
    void* f = nullptr;          // caller's field
    void* G = nullptr;          // [field]: Theta[f^n], then A Theta[f^n]
    void* Y = nullptr;          // [field]: the predictor
    hipStream_t stream = nullptr;
    int dtype = 0;
    long long n = 0;            // values per field
    double tau = 0.0;
    bool poisoned = false;
};

static chasm_status lfail(chasm_status st, const std::string& m)
{
    set_last_error(m);
    return st;
}

static hipError_t combine(chasm_lpc1_s* h, void* x0, const void* x1, void* y, double c, int mode)
{
    const unsigned grid = (unsigned)std::min<long long>((h->n + 255) / 256, 256LL * 64);
    if (h->dtype == CHASM_F64)
        hipLaunchKernelGGL(k_lpc1_combine<double>, dim3(grid), dim3(256), 0, h->stream, static_cast<double*>(x0),
                           static_cast<const double*>(x1), static_cast<double*>(y), h->n, c, mode);
    else
        hipLaunchKernelGGL(k_lpc1_combine<float>, dim3(grid), dim3(256), 0, h->stream, static_cast<float*>(x0),
                           static_cast<const float*>(x1), static_cast<float*>(y), h->n, c, mode);
    return hipGetLastError();
}

extern "C" {

chasm_status chasm_lpc1_create(const chasm_advect_desc* adv, const chasm_theta_desc* th, void* f_dev,
                               void* hip_stream, chasm_lpc1_t* out)
{
    if (!out) return lfail(CHASM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!adv || !th || !f_dev) return lfail(CHASM_EINVAL, "NULL argument");
    if (adv->nbatch != 1 || th->nbatch != 1) return lfail(CHASM_EINVAL, "LPC1 steps one field (nbatch 1)");
    if (adv->flags != 0) return lfail(CHASM_EINVAL, "advection flags must be 0 for LPC1");
    if (adv->dtype != th->dtype) return lfail(CHASM_EINVAL, "advection and theta dtypes differ");
    for (int a = 0; a < 3; ++a)
        if (adv->nx[a] != th->nx[a] || adv->nk[a] != th->nk[a] || adv->x_lo[a] != th->x_lo[a] ||
            adv->x_hi[a] != th->x_hi[a] || adv->k_lo[a] != th->k_lo[a] || adv->k_hi[a] != th->k_hi[a])
            return lfail(CHASM_EINVAL, "advection and theta grids differ");
    if (!(adv->dt > 0) || !std::isfinite(adv->dt)) return lfail(CHASM_EINVAL, "tau (adv->dt) must be finite and > 0");

    chasm_lpc1_s* h = new (std::nothrow) chasm_lpc1_s();
    if (!h) return lfail(CHASM_ENOMEM, "host allocation failed");
    h->f = f_dev;
    h->stream = (hipStream_t)hip_stream;
    h->dtype = adv->dtype;
    h->tau = adv->dt;
    h->n = 1;
    for (int a = 0; a < 3; ++a) h->n *= (long long)adv->nx[a] * adv->nk[a];
    const size_t bytes = (size_t)h->n * (h->dtype == CHASM_F64 ? 8 : 4);
    auto bail = [&](chasm_status s, const std::string& m) {
        chasm_lpc1_destroy(h);
        return lfail(s, m);
    };
    if (hipMalloc(&h->G, bytes) != hipSuccess) return bail(CHASM_ENOMEM, "hipMalloc(theta field) failed");
    if (hipMalloc(&h->Y, bytes) != hipSuccess) return bail(CHASM_ENOMEM, "hipMalloc(predictor) failed");
    chasm_status st = chasm_advect_create(adv, f_dev, hip_stream, &h->adv_f);
    if (st == CHASM_OK) st = chasm_advect_create(adv, h->G, hip_stream, &h->adv_g);
    if (st != CHASM_OK) {
        const std::string m = chasm_advect_last_error();
        return bail(st, "advection: " + m);
    }
    st = chasm_theta_create(th, hip_stream, &h->th);
    if (st != CHASM_OK) {
        const std::string m = chasm_advect_last_error();
        return bail(st, "theta: " + m);
    }
    *out = h;
    return CHASM_OK;
}

chasm_status chasm_lpc1_step(chasm_lpc1_t h, int32_t nsteps)
{
    if (!h) return lfail(CHASM_EINVAL, "handle is NULL");
    if (h->poisoned) return lfail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    if (nsteps < 0) return lfail(CHASM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return CHASM_OK;
    auto dev = [&](hipError_t e, const char* what) {
        h->poisoned = true;
        return lfail(CHASM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e;
    for (int s = 0; s < nsteps; ++s) {
        chasm_status st = chasm_theta_apply(h->th, h->f, h->G);
        if (st == CHASM_OK) st = chasm_advect_step(h->adv_f, 1);
        if (st == CHASM_OK) st = chasm_advect_step(h->adv_g, 1);
        if (st != CHASM_OK) {
            h->poisoned = true;
            return st;
        }
        if ((e = combine(h, h->f, h->G, h->Y, h->tau, 0)) != hipSuccess) return dev(e, "predictor");
        if ((st = chasm_theta_apply(h->th, h->Y, h->Y)) != CHASM_OK) {
            h->poisoned = true;
            return st;
        }
        if ((e = combine(h, h->f, h->G, h->Y, 0.5 * h->tau, 1)) != hipSuccess) return dev(e, "corrector");
    }
    return CHASM_OK;
}

chasm_status chasm_lpc1_destroy(chasm_lpc1_t h)
{
    if (!h) return CHASM_OK;
    if (h->stream) hipStreamSynchronize(h->stream);
    if (h->adv_f) chasm_advect_destroy(h->adv_f);
    if (h->adv_g) chasm_advect_destroy(h->adv_g);
    if (h->th) chasm_theta_destroy(h->th);
    if (h->G) hipFree(h->G);
    if (h->Y) hipFree(h->Y);
    delete h;
    return CHASM_OK;
}

}  // extern "C"

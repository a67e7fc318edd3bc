// chasm_rt.hpp -- runtime-shape path of the characteristic step: any per-axis number
// of nodes N_d, patch length M_d and ghost width g, with the PMBC stencil rows, the
// patch factors and the per-k weights read from device tables built on the host in
// FP64 (Sec. 3.1.2 eqs. 3.4-3.5, step (5); Sec. 3.1.3 eqs. 3.7-3.8).  The compiled
// shapes of chasm_registry.hpp stay the fast path; this path serves every descriptor
// they do not cover, and the Hermite global condition with given end slopes.
#pragma once
#include <hip/hip_runtime.h>

namespace chasm {

// Device tables of one axis (element type T of the kernel: FP64 masters for double
// fields, an FP32 mirror for float fields).
struct RtAxis {
    int N, M, P, MLAST, G;      // nodes, cells per patch, patches, cells of the last patch, window
    int poly3;                  // outer ghost coefficient by a zero fourth difference
    const void* stencil;        // T[(P+1)][2G+1]: interface rows times h, tap t at node I_q - G + t
    const void* bias;           // T[P+1]: given end-slope part of the interface slopes times h
    const void* lu;             // T[2][3][M+1]: (inv, ainv, cp) of the reduced patch system,
                                //   [0] for m = M cells, [1] for m = MLAST
    const int* shift;           // int[nk]: sigma = floor(-alpha)
    const void* w;              // T[nk][4]: weights of the cell taps
};

struct RtJob {
    const void* f;              // field the pass reads
    void* out;                  // field the pass writes (f: in place)
    long long nitems;           // nbatch * nk1 * nk2 * nk3
    int nx[3], nk[3];
    RtAxis ax[3];
};

// Lines per block of a sweep along axis a, or 0 if its LDS tiles do not fit.
int rt_lines_per_block(const RtJob& j, int axis, int elem_bytes);

// One sweep along `axis` for every line of every item; partials (nullable, axis 2
// only): FP64 partial sums of the result, one row per block (rt_rows_per_item rows
// per item, in item order).
hipError_t rt_sweep(const RtJob& j, int axis, int dtype, double* partials, hipStream_t s);
long long rt_rows_per_item(const RtJob& j, int dtype);

// The x3 sweep that ends an observed step, writing the observables' item rows
// (chasm_obs.hpp) in its epilogue; rt_can_observe: the fast form serves this job (else
// the observables take the separate pass).
bool rt_can_observe(const RtJob& j, int dtype);
hipError_t rt_sweep_obs(const RtJob& j, int dtype, double* rows, hipStream_t s);

// Diagnostics of the current field: one partial row per item.
hipError_t rt_reduce(const RtJob& j, int dtype, double* partials, hipStream_t s);

}  // namespace chasm

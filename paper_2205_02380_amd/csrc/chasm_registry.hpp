// chasm_registry.hpp -- the compiled kernel shapes and their launchers.
//
// Every (T, N, M, G) below is compiled: element type T, N nodes per axis (equal on
// all three axes), M cells per patch, G the largest ghost width the kernel's stencil
// window holds (a handle with ghost g uses the smallest G >= g built for its N, M).
#pragma once
#include <hip/hip_runtime.h>

namespace chasm {

struct JobDev;

// partials: FP64 block partials (nullptr: no reduction).  Grids are derived from
// job.nitems.  Returns the launch status.
using LaunchFn = hipError_t (*)(const JobDev& job, double* partials, hipStream_t stream);

struct KernelSet {
    int dtype;              // 0 float, 1 double
    int N, M, G;
    LaunchFn cube;          // nullptr when the x-cube does not fit in LDS
    LaunchFn slab_x1;
    LaunchFn slab_x1x2;
    LaunchFn pencil_x2;
    LaunchFn pencil_x3;
    LaunchFn reduce;        // diagnostics of the current field (one partial row per item)
    int cube_rows;          // partial rows per item written by cube (1)
    int pencil_rows;        // partial rows per item written by pencil_x3
};

template <typename T, int N, int M, int G>
const KernelSet* kernel_set();

// (T, N, M, G) shapes, grouped by (N, dtype): one compilation unit per group.
// FP64 is built for the grids the plain FP64 form and the FP64 parity cases use.
#define CHASM_SHAPES_N8_F32(X) X(float, 8, 2, 7) X(float, 8, 4, 7) X(float, 8, 8, 7)
#define CHASM_SHAPES_N8_F64(X) X(double, 8, 2, 7) X(double, 8, 4, 7) X(double, 8, 8, 7)
#define CHASM_SHAPES_N16_F32(X) X(float, 16, 4, 8) X(float, 16, 8, 8) X(float, 16, 16, 8) X(float, 16, 8, 15)
#define CHASM_SHAPES_N16_F64(X) X(double, 16, 4, 8) X(double, 16, 8, 8) X(double, 16, 16, 8) X(double, 16, 8, 15)
#define CHASM_SHAPES_N24_F32(X) X(float, 24, 8, 8) X(float, 24, 12, 8)
#define CHASM_SHAPES_N24_F64(X) X(double, 24, 8, 8) X(double, 24, 12, 8)
#define CHASM_SHAPES_N32_F32(X) X(float, 32, 8, 8) X(float, 32, 16, 8)
#define CHASM_SHAPES_N32_F64(X) X(double, 32, 8, 8) X(double, 32, 16, 8)
#define CHASM_SHAPES_N48_F32(X) X(float, 48, 8, 8) X(float, 48, 12, 8) X(float, 48, 16, 8)
#define CHASM_SHAPES_N64_F32(X) X(float, 64, 8, 8) X(float, 64, 16, 8)
#define CHASM_SHAPES(X)                                                                                   \
    CHASM_SHAPES_N8_F32(X) CHASM_SHAPES_N8_F64(X) CHASM_SHAPES_N16_F32(X) CHASM_SHAPES_N16_F64(X)          \
    CHASM_SHAPES_N24_F32(X) CHASM_SHAPES_N24_F64(X) CHASM_SHAPES_N32_F32(X) CHASM_SHAPES_N32_F64(X)        \
    CHASM_SHAPES_N48_F32(X) CHASM_SHAPES_N64_F32(X)

}  // namespace chasm

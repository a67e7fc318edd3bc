// chasm_registry.hpp -- the compiled kernel shapes and their launchers.
//
// Every (T, N, M, G, CL) below is compiled: element type T, N nodes per axis (equal
// on all three axes), M cells per patch, ghost width G, closure CL (0 the paper's
// PMBC, 1 the cubic-exact variant).  The stencil rows and patch factors of a shape
// are compile-time constants, so a handle needs an exact match.
#pragma once
#include <hip/hip_runtime.h>

namespace chasm {

struct Work;

// partials: FP64 block partials (nullptr: no reduction).  Grids are derived from the
// work list's item count.  Returns the launch status.
using LaunchFn = hipError_t (*)(const Work& w, double* partials, hipStream_t stream);

struct KernelSet {
    int dtype;              // 0 float, 1 double
    int N, M, G, CL;
    int tile;               // launch-shape variant (chasm_launch.hpp)
    LaunchFn cube;          // nullptr when the x-cube does not fit in LDS
    // x3-slab passes by sweep sequence: [0] x1, [1] x1 x2, [2] x2 x1 x1 x2 (partials
    // after the first x1), [3] x2 x1 (partials after x1)
    LaunchFn slab[4];
    LaunchFn pencil_x2;
    LaunchFn pencil_x3;     // partials after the x3 sweep
    LaunchFn pencil_x3x3;   // two x3 sweeps, partials after the first
    LaunchFn pencil_x3_obs; // one x3 sweep writing the observables' item rows (chasm_obs.hpp)
    LaunchFn reduce;        // diagnostics of the current field (one partial row per item)
    int cube_rows;          // partial rows per item written by cube (1)
    int pencil_rows;        // partial rows per item written by the x3 pencils
    int slab_rows;          // partial rows per item written by the slab passes
};

template <typename T, int N, int M, int G, int CL, int TILE>
const KernelSet* kernel_set();

// (T, N, M, G, CL) shapes, grouped by (N, dtype); the build compiles each shape in a
// generated unit of its own.
// FP32: the benchmark and serving grids, the autotuner's patch x ghost sweep for the
// 32^3 / 48^3 / 64^3 grids, and the test shapes.  FP64: the plain FP64 form (also at
// the 48^3 and 64^3 grids) and the FP64 parity cases.
#define CHASM_SHAPES_N8_F32(X) X(float, 8, 2, 1, 0) X(float, 8, 4, 3, 0) X(float, 8, 8, 7, 0) X(float, 8, 4, 3, 2)
#define CHASM_SHAPES_N8_F64(X) X(double, 8, 2, 1, 0) X(double, 8, 4, 3, 0) X(double, 8, 8, 7, 0) X(double, 8, 4, 3, 2)
#define CHASM_SHAPES_N16_F32(X)                                                                        \
    X(float, 16, 8, 4, 0) X(float, 16, 8, 4, 1) X(float, 16, 8, 6, 0) X(float, 16, 4, 8, 0)              \
    X(float, 16, 8, 15, 0) X(float, 16, 16, 5, 0) X(float, 16, 8, 4, 2)
#define CHASM_SHAPES_N16_F64(X)                                                                        \
    X(double, 16, 8, 4, 0) X(double, 16, 8, 4, 1) X(double, 16, 8, 6, 0) X(double, 16, 4, 8, 0)          \
    X(double, 16, 8, 15, 0) X(double, 16, 16, 5, 0) X(double, 16, 8, 4, 2)
#define CHASM_SHAPES_N24_F32(X) X(float, 24, 8, 6, 0) X(float, 24, 12, 6, 0)
#define CHASM_SHAPES_N24_F64(X) X(double, 24, 8, 6, 0) X(double, 24, 12, 6, 0)
#define CHASM_SHAPES_N32_F32(X)                                                                        \
    X(float, 32, 8, 4, 0) X(float, 32, 8, 6, 0) X(float, 32, 8, 8, 0) X(float, 32, 16, 4, 0)             \
    X(float, 32, 16, 6, 0) X(float, 32, 16, 8, 0) X(float, 32, 8, 6, 2)
#define CHASM_SHAPES_N32_F64(X) X(double, 32, 8, 6, 0) X(double, 32, 16, 8, 0)
#define CHASM_SHAPES_N48_F32(X)                                                                        \
    X(float, 48, 8, 4, 0) X(float, 48, 8, 6, 0) X(float, 48, 8, 8, 0) X(float, 48, 12, 4, 0)             \
    X(float, 48, 12, 6, 0) X(float, 48, 12, 8, 0) X(float, 48, 16, 4, 0) X(float, 48, 16, 6, 0)          \
    X(float, 48, 16, 8, 0)
#define CHASM_SHAPES_N64_F32(X)                                                                        \
    X(float, 64, 8, 4, 0) X(float, 64, 8, 6, 0) X(float, 64, 8, 8, 0) X(float, 64, 16, 4, 0)             \
    X(float, 64, 16, 6, 0) X(float, 64, 16, 8, 0)
#define CHASM_SHAPES_N48_F64(X) X(double, 48, 16, 8, 0)
#define CHASM_SHAPES_N64_F64(X) X(double, 64, 16, 8, 0)
// Shapes compiled in the tile variants 1 and 2 as well (the autotuner's tile-shape
// axis): the 48^3 FP32 shapes of its patch x ghost sweep, and the 64^3 FP32 shape of
// the one-GPU-share grid.
#define CHASM_TILED_SHAPES(X) CHASM_SHAPES_N48_F32(X) X(float, 64, 16, 8, 0)
constexpr int kTiles = 3;
#define CHASM_SHAPES(X)                                                                                   \
    CHASM_SHAPES_N8_F32(X) CHASM_SHAPES_N8_F64(X) CHASM_SHAPES_N16_F32(X) CHASM_SHAPES_N16_F64(X)          \
    CHASM_SHAPES_N24_F32(X) CHASM_SHAPES_N24_F64(X) CHASM_SHAPES_N32_F32(X) CHASM_SHAPES_N32_F64(X)        \
    CHASM_SHAPES_N48_F32(X) CHASM_SHAPES_N48_F64(X) CHASM_SHAPES_N64_F32(X) CHASM_SHAPES_N64_F64(X)

}  // namespace chasm

// chasm_launch.hpp -- launch shapes and launchers of the kernel templates.
// Included only by the instantiation units (inst_n*.hip).
#pragma once
#include "chasm_kernels.hpp"
#include "chasm_registry.hpp"

namespace chasm {

// LDS available to one work-group on gfx950.
constexpr size_t kLdsBytes = 160 * 1024;

// Launch shapes of (T, N) for tile variant TILE (the autotuner's tile-shape axis; the
// kernels' arithmetic per line does not depend on it, so results are bitwise equal):
//   0  the defaults below;
//   1  twice the x3-slabs per slab block, 128 lines per pencil block;
//   2  the default slab block, 384 (N = 48) or 512 (N = 64) lines per pencil block.
// Variants 1 and 2 are compiled for the FP32 48^3 and 64^3 shapes only.
template <typename T, int N, int TILE = 0>
struct Launch {
    static_assert(TILE == 0 || N == 48 || N == 64, "tile variants exist for N = 48 and 64");
    // Whole x-cube in LDS (rows padded to N+1) plus the block-sum scratch.
    static constexpr bool cube_fits = (size_t)N * N * (N + 1) * sizeof(T) + 1024 <= kLdsBytes;
    // threads per cube block: a multiple of N whose planes-per-round NT/N divide N;
    // FP32 uses one line per thread per sweep up to N = 32 (4 waves per SIMD)
    static constexpr int cube_nt =
        N <= 8 ? 64 : (N <= 16 ? 256 : (N <= 24 ? (sizeof(T) == 4 ? 576 : 192) : 1024));
    // x3-slabs per slab block: S*N threads, a multiple of 64, S | N.
    static constexpr int slab_s0 = N == 8 ? 8 : (N == 16 ? 4 : (N == 24 ? 8 : (N == 32 ? 2 : (N == 48 ? 4 : 1))));
    static constexpr int slab_s = TILE == 1 ? 2 * slab_s0 : slab_s0;
    // lines per pencil block: a multiple of 64 dividing N*N.
    static constexpr int pencil_nt0 = N == 8 ? 64 : (N == 24 ? 192 : 256);
    static constexpr int pencil_nt = TILE == 1 ? 128 : (TILE == 2 ? (N == 48 ? 384 : 512) : pencil_nt0);
    // Slab passes keep the next unit's loads in flight in VGPRs (see k_slab) where a
    // line is at most 256 bytes, except the four-sweep pass (SLAB_X2X1X1X2), whose VGPRs
    // go to the register-resident x1 pair instead (see k_slab).  At N = 64 (one 16 KB
    // plane per 64-thread block, occupancy bound by LDS at nine planes per CU) the
    // prefetch had taken that pass from 14.9 to 13.7 ms on the 64^3 x 32^3 grid with the
    // x1 pair through LDS; the register pair without the prefetch is faster again (13.0
    // -> 12.9 ms per step with per-step reductions), and with the prefetch as well it
    // needs 256 VGPRs (one wave per SIMD).  Streamed (nontemporal) field accesses at
    // N = 64 (slab_cpol) gain a further 2 %; at N = 48 default caching is faster.
    static constexpr bool slab_pre = sizeof(T) * N <= 256;
    static constexpr int slab_cpol = N == 64 ? kCpolStream : 0;
    static constexpr int reduce_nt = 256;
};

// Resident blocks of kernel K on the current device (CUs x blocks per CU), cached per
// device; one cache per kernel instantiation.
template <auto K>
int resident_blocks(int threads)
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cache[dev] == 0) {
        int ncu = 0, per = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, K, threads, 0) != hipSuccess) return 0;
        cache[dev] = ncu * (per > 0 ? per : 1);
    }
    return cache[dev];
}

// Persistent launch: one block per resident slot, at most one per unit of work.
template <auto K, typename... A>
hipError_t launch_persistent(int threads, long long units, hipStream_t s, A... args)
{
    const long long res = resident_blocks<K>(threads);
    const unsigned grid = (unsigned)(res > 0 && res < units ? res : units);
    hipLaunchKernelGGL(K, dim3(grid), dim3(threads), 0, s, args...);
    return hipGetLastError();
}

template <typename T, int N, int M, int G, int CL>
hipError_t launch_cube(const Work& w, double* partials, hipStream_t s)
{
    using Lc = Launch<T, N>;
    if constexpr (Lc::cube_fits) {
        constexpr int NT = Lc::cube_nt;
        const long long items = w.first[w.njobs];
        return partials ? launch_persistent<k_cube<T, N, M, G, CL, NT, true>>(NT, items, s, w, partials)
                        : launch_persistent<k_cube<T, N, M, G, CL, NT, false>>(NT, items, s, w, partials);
    } else {
        return hipErrorInvalidConfiguration;
    }
}

template <typename T, int N, int M, int G, int CL, int MODE, int TILE>
hipError_t launch_slab(const Work& w, double* partials, hipStream_t s)
{
    using Lc = Launch<T, N, TILE>;
    constexpr int S = Lc::slab_s;
    constexpr bool PRE = MODE != SLAB_X2X1X1X2 && Lc::slab_pre;
    constexpr int CP = Lc::slab_cpol;
    const long long units = w.first[w.njobs] * (N / S);
    if constexpr (MODE == SLAB_X2X1X1X2 || MODE == SLAB_X2X1) {
        if (partials)
            return launch_persistent<k_slab<T, N, M, G, CL, S, MODE, PRE, true, CP>>(S * N, units, s, w, partials);
    }
    return launch_persistent<k_slab<T, N, M, G, CL, S, MODE, PRE, false, CP>>(S * N, units, s, w, nullptr);
}

template <typename T, int N, int M, int G, int CL, int AXIS, int NSW, int TILE>
hipError_t launch_pencil(const Work& w, double* partials, hipStream_t s)
{
    using Lc = Launch<T, N, TILE>;
    constexpr int NT = Lc::pencil_nt;
    const unsigned grid = (unsigned)(w.first[w.njobs] * (N * N / NT));
    if (AXIS == 2 && partials)
        hipLaunchKernelGGL((k_pencil<T, N, M, G, CL, NT, AXIS, NSW, AXIS == 2>), dim3(grid), dim3(NT), 0, s, w,
                           partials);
    else
        hipLaunchKernelGGL((k_pencil<T, N, M, G, CL, NT, AXIS, NSW, false>), dim3(grid), dim3(NT), 0, s, w, partials);
    return hipGetLastError();
}

// The x3 sweep that ends an observed step: rows = the observables' item rows.
template <typename T, int N, int M, int G, int CL, int TILE>
hipError_t launch_pencil_obs(const Work& w, double* rows, hipStream_t s)
{
    using Lc = Launch<T, N, TILE>;
    constexpr int NT = Lc::pencil_nt;
    const unsigned grid = (unsigned)(w.first[w.njobs] * (N * N / NT));
    hipLaunchKernelGGL((k_pencil<T, N, M, G, CL, NT, 2, 1, false, true>), dim3(grid), dim3(NT), 0, s, w, rows);
    return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_reduce(const Work& w, double* partials, hipStream_t s)
{
    using Lc = Launch<T, N>;
    hipLaunchKernelGGL((k_reduce_field<T, N, Lc::reduce_nt>), dim3((unsigned)w.first[w.njobs]), dim3(Lc::reduce_nt), 0,
                       s, w, partials);
    return hipGetLastError();
}

template <typename T, int N, int M, int G, int CL, int TILE>
const KernelSet* kernel_set()
{
    using Lc = Launch<T, N, TILE>;
    static const KernelSet ks = {
        sizeof(T) == 8 ? 1 : 0,
        N,
        M,
        G,
        CL,
        TILE,
        // the cube schedule has one launch shape (tile 0)
        (TILE == 0 && Lc::cube_fits) ? &launch_cube<T, N, M, G, CL> : nullptr,
        {&launch_slab<T, N, M, G, CL, SLAB_X1, TILE>, &launch_slab<T, N, M, G, CL, SLAB_X1X2, TILE>,
         &launch_slab<T, N, M, G, CL, SLAB_X2X1X1X2, TILE>, &launch_slab<T, N, M, G, CL, SLAB_X2X1, TILE>},
        &launch_pencil<T, N, M, G, CL, 1, 1, TILE>,
        &launch_pencil<T, N, M, G, CL, 2, 1, TILE>,
        &launch_pencil<T, N, M, G, CL, 2, 2, TILE>,
        &launch_pencil_obs<T, N, M, G, CL, TILE>,
        &launch_reduce<T, N>,
        1,
        N * N / Lc::pencil_nt,
        N / Lc::slab_s,
    };
    return &ks;
}

#define CHASM_INSTANTIATE(T, N, M, G, CL) template const KernelSet* kernel_set<T, N, M, G, CL, 0>();
#define CHASM_INSTANTIATE_TILE(T, N, M, G, CL, TILE) template const KernelSet* kernel_set<T, N, M, G, CL, TILE>();

}  // namespace chasm

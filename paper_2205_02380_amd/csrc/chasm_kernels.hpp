// chasm_kernels.hpp -- gfx950 kernels of the characteristic (spatial-advection)
// step of the CHASM scheme (arXiv:2205.02380, Sec. 3), f(x,k) <- f(x - k dt, k).
//
// Field layout: f[b][k3][k2][k1][x3][x2][x1], x1 fastest; one "item" is the x-cube of
// one (b, k) pair (N^3 contiguous values).  The three axis sweeps of a step
// (eqs. 3.11-3.12 factored axis by axis, order x1, x2, x3) are independent per item,
// because the shift alpha_d = k_d dt / h_d depends on k only.
//
// Kernels (each reads the job's field f and writes its destination `out` once per
// launch; out == f is in place, out != f runs the pass out of place into a buffer of
// the same shape):
//   k_cube    all three sweeps of one item with the whole x-cube in LDS
//             (N^2 (N+1) values, rows padded to N+1 so x1-, x2- and x3-lines are
//             bank-conflict free): 8 B/point-update in FP32.
//   k_slab    x1 and x2 sweeps (see SlabMode) on S x3-slabs (N x N) held in LDS;
//             persistent, with the next unit's loads in flight.
//   k_pencil  one or two x2 or x3 sweeps; each lane holds one whole line in VGPRs,
//             lanes of a wave hold neighbouring x1 columns, so every load and store
//             of the wave is a contiguous run of x1.
//   k_reduce_field, k_finalize: FP64 diagnostics (mass, L2, first moments).
// Reductions can be fused into the last sweep of a step; every block writes its
// own FP64 partials and k_finalize sums them in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chasm_line.hpp"
#include "chasm_obs.hpp"

namespace chasm {

struct AxisTabDev {
    const int* shift;      // int[nk]   sigma = floor(-alpha(k))
    const void* w;         // T[nk][4]  shift weights
};

struct JobDev {
    void* f;               // field base the pass reads
    void* out;             // base the pass writes: f (in place) or a field of the same shape
    int reverse;           // k_cube visits this job's items last to first
    long long nitems;      // nbatch * nk1 * nk2 * nk3
    int nk[3];
    AxisTabDev ax[3];
};

// The jobs of one launch, passed by value in the kernel arguments: items of job j are
// the global items [first[j], first[j+1]).  One handle is a one-job list; several
// handles with the same kernels share a launch (continuous batching).
constexpr int kMaxJobs = 24;
struct Work {
    int njobs;
    long long first[kMaxJobs + 1];
    JobDev jobs[kMaxJobs];
};

// Job of a global item (uniform across the block) and the item's index in that job.
__device__ __forceinline__ const JobDev& job_of(const Work& w, long long item, long long& local)
{
    int j = 0;
    while (j + 1 < w.njobs && item >= w.first[j + 1]) ++j;
    local = item - w.first[j];
    return w.jobs[j];
}

// Number of FP64 partials written per block when reducing.
constexpr int NRED = 8;

template <typename T>
struct Vec16;
template <>
struct Vec16<float> { using type = float4; static constexpr int n = 4; };
template <>
struct Vec16<double> { using type = double2; static constexpr int n = 2; };

template <typename T>
__device__ __forceinline__ T vget(const typename Vec16<T>::type& v, int i);
template <>
__device__ __forceinline__ float vget<float>(const float4& v, int i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
template <>
__device__ __forceinline__ double vget<double>(const double2& v, int i) { return i == 0 ? v.x : v.y; }

template <typename T>
__device__ __forceinline__ void vset(typename Vec16<T>::type& v, int i, T x);
template <>
__device__ __forceinline__ void vset<float>(float4& v, int i, float x)
{
    if (i == 0) v.x = x; else if (i == 1) v.y = x; else if (i == 2) v.z = x; else v.w = x;
}
template <>
__device__ __forceinline__ void vset<double>(double2& v, int i, double x)
{
    if (i == 0) v.x = x; else v.y = x;
}

// Raw buffer access: a per-wave resource over [base, base + bytes), a per-lane byte
// offset (VGPR) and a uniform byte offset (SGPR), so a strided line needs no
// per-element 64-bit address registers.  Out-of-range accesses load 0 and drop
// stores (hardware range check against the resource size).
// Cache policy of the field's buffer loads and stores (the aux operand of the buffer
// intrinsics: 2 sets the nontemporal bit, 0 is default caching).
//  - k_pencil streams (kCpolStream): every field value is read once and written once
//    per launch; measured 8 % faster on the C3 x3 pass than default caching.
//  - k_cube caches (kCpolCube): consecutive steps visit the items in opposite orders,
//    so the cubes a step stores last are loaded first by the next step and can still
//    be in the memory-side cache; streamed accesses do not allocate there.  Measured
//    on C2 (537 MB field): 0.194 ms per step streamed in either order, 0.181 ms with
//    default caching and alternating order.
//  - k_slab takes its policy as a template argument (see Launch::slab_cpol): streamed
//    at N = 64, default caching at N = 48.
// Results are bitwise equal under every policy.
constexpr int kCpolStream = 2;
constexpr int kCpolCube = 0;

struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ Buf(const void* base, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000))
    {
    }
    template <typename T, int CP = kCpolStream>
    __device__ __forceinline__ T load(uint32_t voff, uint32_t soff) const
    {
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, CP));
        } else {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, CP));
        }
    }
    template <typename T, int CP>
    __device__ __forceinline__ typename Vec16<T>::type load16(uint32_t voff, uint32_t soff) const
    {
        return __builtin_bit_cast(typename Vec16<T>::type,
                                  __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, CP));
    }
    template <typename T, int CP>
    __device__ __forceinline__ void store16(const typename Vec16<T>::type& x, uint32_t voff, uint32_t soff) const
    {
        using I4 = int __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(I4, x), r, (int)voff, (int)soff, CP);
    }
    template <typename T, int CP = kCpolStream>
    __device__ __forceinline__ void store(T x, uint32_t voff, uint32_t soff) const
    {
        if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, x), r, (int)voff, (int)soff, CP);
        } else {
            using I2 = int __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(I2, x), r, (int)voff, (int)soff, CP);
        }
    }
};

// k indices of an item (items < 2^31 and k-points per field < 2^31: validated on the host).
__device__ __forceinline__ void item_k(const JobDev& job, long long item, int ik[3])
{
    const unsigned nk0 = (unsigned)job.nk[0], nk1 = (unsigned)job.nk[1];
    const unsigned nkp = nk0 * nk1 * (unsigned)job.nk[2];
    const unsigned kf = (unsigned)item % nkp;
    ik[0] = (int)(kf % nk0);
    ik[1] = (int)((kf / nk0) % nk1);
    ik[2] = (int)(kf / (nk0 * nk1));
}

// Tables are read-only for the whole kernel: read them through the constant address
// space, which lets the compiler use scalar loads into SGPRs.
template <typename T>
using cptr = const T __attribute__((address_space(4)))*;

template <typename T>
__device__ __forceinline__ AxisCoef<T> axis_coef(const JobDev& job, int d, int ik, int& sigma)
{
    const AxisTabDev& a = job.ax[d];
    const cptr<T> w = (cptr<T>)(a.w) + 4 * ik;
    AxisCoef<T> c;
    c.w0 = w[0];
    c.w1 = w[1];
    c.w2 = w[2];
    c.w3 = w[3];
    sigma = ((const int __attribute__((address_space(4)))*)(a.shift))[ik];
    return c;
}

// One DPP lane move of a double (both halves, every lane written).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum NV doubles over the block; thread 0 ends up with the totals in acc.
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV])
{
    __shared__ double red[NT / 64][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        // within each row of 16 lanes by DPP moves (VALU): pairs, quads, then the
        // half-row and row mirrors, which pair lanes of groups already summed; across
        // rows by two lane permutes
        double x = acc[v];
        x += dpp_f64<0xB1>(x);    // quad_perm [1,0,3,2]
        x += dpp_f64<0x4E>(x);    // quad_perm [2,3,0,1]
        x += dpp_f64<0x141>(x);   // row_half_mirror
        x += dpp_f64<0x140>(x);   // row_mirror
        x += __shfl_xor(x, 16, 64);
        x += __shfl_xor(x, 32, 64);
        acc[v] = x;
    }
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    if (NT > 64) {
        if (ln == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) red[wv][v] = acc[v];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double s = 0.0;
                for (int w = 0; w < NT / 64; ++w) s += red[w][v];
                acc[v] = s;
            }
        }
    }
}

// Block partials: [sum f, sum f^2, sum i1 f, sum i2 f, sum i3 f, sum ik1 f, sum ik2 f, sum ik3 f].
template <int NT>
__device__ __forceinline__ void write_partials(double (&acc)[5], const int ik[3], double* __restrict__ out)
{
    block_sum<NT, 5>(acc);
    if (threadIdx.x == 0) {
        out[0] = acc[0];
        out[1] = acc[1];
        out[2] = acc[2];
        out[3] = acc[3];
        out[4] = acc[4];
        out[5] = ik[0] * acc[0];
        out[6] = ik[1] * acc[0];
        out[7] = ik[2] * acc[0];
    }
}

// ---------------------------------------------------------------------------
// Whole x-cube in LDS: x1, x2 and x3 sweeps of one item at a time.
//
// Persistent: each block walks items blockIdx.x, blockIdx.x + gridDim.x, ...  An item
// enters LDS in rounds of PL = NT/N x3-planes; the x1 and x2 sweeps only couple nodes
// within a plane, so they run on each round as soon as it lands, while the next
// round -- or, after the last round, the next item's first round -- is already in
// flight into VGPRs (N/VW 16-byte buffer loads per lane).  The x3 sweep then runs on
// the whole cube and the result streams out, with the FP64 partials when asked for.
template <typename T, int N, int M, int G, int CL, int NT, bool RED>
__global__ __launch_bounds__(NT) void k_cube(const Work w, double* __restrict__ partials)
{
    constexpr int PX = N + 1;
    constexpr int VW = Vec16<T>::n;
    constexpr int PL = NT / N;                    // planes per round
    constexpr int ROUNDS = N / PL;
    constexpr int RV = N / VW;                    // 16-byte vectors per lane per round
    constexpr int NV = N * N * N / VW;            // 16-byte vectors per cube
    constexpr int RSTEP = NT * VW / N;            // cube rows between a lane's vectors
    constexpr uint32_t CUBE_BYTES = (uint32_t)(N * N * N * sizeof(T));
    static_assert(NT % N == 0 && N % PL == 0 && N % VW == 0 && NV % NT == 0 && (NT * VW) % N == 0,
                  "bad cube tiling");
    using V = typename Vec16<T>::type;
    __shared__ T lds[N * N * PX];

    // Per-lane bases; every other index below is a compile-time offset from them.
    // tid is re-derived inside the item loop through an opaque copy, so the bases are
    // recomputed per item instead of being pinned in registers for the whole loop.
    unsigned tid = threadIdx.x;
    V pre[RV];
    const long long total = w.first[w.njobs];
    // Item `it` of the visiting order: its job and index in the job (reversed jobs are
    // visited last item first).
    auto locate = [&](long long it, long long& local) -> const JobDev& {
        const JobDev& jb = job_of(w, it, local);
        if (jb.reverse) local = jb.nitems - 1 - local;
        return jb;
    };
    auto cube_of = [&](long long it) {
        long long local;
        const JobDev& jb = locate(it, local);
        return static_cast<T*>(jb.f) + local * (long long)(N * N * N);
    };
    auto fetch = [&](long long it, int round) {
        const Buf b(cube_of(it), CUBE_BYTES);
        static_for<0, RV>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            pre[q] = b.template load16<T, kCpolCube>(tid * 16u, (uint32_t)((round * RV + q) * NT * 16));
        });
    };

    // Round r of an item: LDS rows of planes [r*PL, (r+1)*PL) from pre[].
    auto fill = [&](int r) {
        const unsigned vbase = (tid * VW / N) * PX + (tid * VW) % N;
        static_for<0, RV>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            T* dst = lds + vbase + (unsigned)((r * RV + q) * RSTEP * PX);
#pragma unroll
            for (int i = 0; i < VW; ++i) dst[i] = vget<T>(pre[q], i);
        });
    };

    long long item = blockIdx.x;
    if (item >= total) return;
    fetch(item, 0);
    fill(0);
    // The loop is rotated: an item's first round is written to LDS at the end of the
    // previous iteration.
    for (;;) {
        tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        // vector v = q*NT + tid of the cube holds elements (q*NT + tid)*VW.. : its row is
        // q*RSTEP + tid*VW/N and its first x1 is tid*VW % N
        const unsigned vbase = (tid * VW / N) * PX + (tid * VW) % N;
        const unsigned plane_t = tid / N, lane_t = tid % N;
        const long long next = item + gridDim.x;
        long long local;
        const JobDev& job = locate(item, local);
        int ik[3];
        item_k(job, local, ik);
        int sig0, sig1;
        const auto k0 = axis_coef<T>(job, 0, ik[0], sig0);
        const auto k1 = axis_coef<T>(job, 1, ik[1], sig1);

#pragma unroll 1
        for (int r = 0; r < ROUNDS; ++r) {
            if (r > 0) fill(r);
            __syncthreads();
            if (r + 1 < ROUNDS) fetch(item, r + 1);
            else if (next < total) fetch(next, 0);
            const unsigned plane = r * PL + plane_t;
            {   // x1: row (x2 = lane_t) of this thread's plane
                T* row = lds + (plane * N + lane_t) * PX;
                dispatch_sigma(sig0, [&](auto sc) {
                    T v[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i] = row[i];
                    advect_line<T, N, M, G, CL, decltype(sc)::value>(v, k0, sig0, [&](int j, T x) { row[j] = x; });
                });
            }
            __syncthreads();
            {   // x2: column (x1 = lane_t) of this thread's plane
                T* col = lds + plane * N * PX + lane_t;
                dispatch_sigma(sig1, [&](auto sc) {
                    T v[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i] = col[i * PX];
                    advect_line<T, N, M, G, CL, decltype(sc)::value>(v, k1, sig1,
                                                                       [&](int j, T x) { col[j * PX] = x; });
                });
            }
        }
        __syncthreads();
        {   // x3 over the whole cube: lines (x1, x2) = (l % N, l / N), l = tid + q*NT
            int sig2;
            const auto k2 = axis_coef<T>(job, 2, ik[2], sig2);
            const unsigned lbase = plane_t * PX + lane_t;
            dispatch_sigma(sig2, [&](auto sc) {
                constexpr int SIG = decltype(sc)::value;
                static_for<0, N * N / NT>([&](auto qc) {
                    T* line = lds + lbase + (unsigned)(decltype(qc)::value * PL * PX);
                    T v[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i] = line[i * N * PX];
                    advect_line<T, N, M, G, CL, SIG>(v, k2, sig2, [&](int j, T x) { line[j * N * PX] = x; });
                });
            });
        }
        __syncthreads();

        // Read the finished cube out of LDS; it is stored only after the next item's
        // first round has been written to LDS (below), so no store is ever issued
        // between a prefetch load and the point where its data is consumed.
        V out[NV / NT];
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        const unsigned row_t = tid * VW / N, x1_t = (tid * VW) % N;
        static_for<0, NV / NT>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const T* src = lds + vbase + (unsigned)(q * RSTEP * PX);
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < VW; ++i) {
                const T y = src[i];
                vset<T>(out[q], i, y);
                if constexpr (RED) {
                    const double yd = (double)y;
                    sum += yd;
                    acc[1] = fma(yd, yd, acc[1]);
                    acc[2] = fma((double)i, yd, acc[2]);
                }
            }
            if constexpr (RED) {
                const unsigned row = q * RSTEP + row_t;
                acc[0] += sum;
                acc[3] = fma((double)(row % N), sum, acc[3]);
                acc[4] = fma((double)(row / N), sum, acc[4]);
            }
        });
        if constexpr (RED) {
            acc[2] = fma((double)x1_t, acc[0], acc[2]);   // sum (x1_t + i) f
            long long local0;
            job_of(w, item, local0);
            write_partials<NT>(acc, ik, partials + (item - local0 + local) * NRED);   // row of the stored item
        }
        __syncthreads();
        if (next < total) fill(0);
        const Buf b(static_cast<T*>(job.out) + local * (long long)(N * N * N), CUBE_BYTES);
        static_for<0, NV / NT>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            b.template store16<T, kCpolCube>(out[q], tid * 16u, (uint32_t)(q * NT * 16));
        });
        if (next >= total) break;
        item = next;
    }
}

// ---------------------------------------------------------------------------
// Sweep sequences of k_slab (applied to every x3-slab of a unit, left to right):
//   SLAB_X1        x1                 (first launch of the three-launch schedule)
//   SLAB_X1X2      x1 x2              (first pass of a step)
//   SLAB_X2X1X1X2  x2 x1 | x1 x2      (the end of one step and the start of the next)
//   SLAB_X2X1      x2 x1              (the end of the last step of a call)
// Consecutive steps of a multi-step call alternate the sweep order, x1 x2 x3 then
// x3 x2 x1: the three axis operators act on different indices of the tensor-product
// spline (eqs. 3.11-3.12) and commute exactly, so the order changes only the rounding.
// Adjacent sweeps along the same axes then share a pass: K steps take K + 1 passes
// (slab, pencil, slab, ...), one read and one write of the field per pass.
enum SlabMode { SLAB_X1 = 0, SLAB_X1X2 = 1, SLAB_X2X1X1X2 = 2, SLAB_X2X1 = 3 };

// S x3-slabs (N x N each) per block in LDS, block = S*N threads (one line each per
// sweep).  Persistent over units of S consecutive slabs of one item.  PRE: the next
// unit's 16-byte loads are in flight in VGPRs while this unit is swept and stored
// (otherwise a unit is loaded when its turn comes, and other resident blocks hide the
// latency).  Units are disjoint, so in place a prefetch never reads what another unit
// writes.
// RED: FP64 partials of the field after the sweep that completes a step (the first
// x1 sweep of SLAB_X2X1X1X2, the x1 sweep of SLAB_X2X1), one row per unit.
template <typename T, int N, int M, int G, int CL, int S, int MODE, bool PRE, bool RED, int CP = 0>
__global__ __launch_bounds__(S * N) void k_slab(const Work w, double* __restrict__ partials)
{
    constexpr int PX = N + 1;
    constexpr int NT = S * N;
    constexpr int VW = Vec16<T>::n;
    constexpr int RV = S * N * N / VW / NT;        // 16-byte vectors per lane per unit
    static_assert(N % VW == 0 && N % S == 0 && (S * N * N / VW) % NT == 0, "bad slab shape");
    static_assert(!RED || MODE == SLAB_X2X1X1X2 || MODE == SLAB_X2X1, "no step ends in this pass");
    using V = typename Vec16<T>::type;
    __shared__ T lds[S * N * PX];

    constexpr int BPI = N / S;                     // units per item
    const long long units = w.first[w.njobs] * BPI;
    long long u = blockIdx.x;
    if (u >= units) return;
    V pre[RV];
    constexpr uint32_t UNIT_BYTES = (uint32_t)(S * N * N * sizeof(T));
    auto fetch = [&](long long uu) {
        long long it;
        const JobDev& jb = job_of(w, uu / BPI, it);
        const Buf b(static_cast<const T*>(jb.f) + it * (long long)(N * N * N) + (long long)(uu % BPI) * S * N * N,
                    UNIT_BYTES);
        static_for<0, RV>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            pre[q] = b.template load16<T, CP>(threadIdx.x * 16u, (uint32_t)(q * NT * 16));
        });
    };
    if constexpr (PRE) fetch(u);
    for (;;) {
        if constexpr (!PRE) fetch(u);
        static_for<0, RV>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int e = q * NT + threadIdx.x;
            const int row = (e * VW) / N, x1 = (e * VW) % N;
#pragma unroll
            for (int i = 0; i < VW; ++i) lds[row * PX + x1 + i] = vget<T>(pre[q], i);
        });
        __syncthreads();
        const long long next = u + gridDim.x;
        if constexpr (PRE) {
            if (next < units) fetch(next);
        }

        long long item;
        const JobDev& job = job_of(w, u / BPI, item);
        const int slab0 = (int)(u % BPI) * S;
        int ik[3];
        item_k(job, item, ik);
        T* out_ptr = static_cast<T*>(job.out) + item * (long long)(N * N * N) + (long long)slab0 * N * N;
        const int slab_t = threadIdx.x / N, col_t = threadIdx.x % N;
        double s = 0.0, s2 = 0.0, sj = 0.0;        // partial sums of this thread's row (RED)
        auto tally = [&](int j, T x) {
            if constexpr (RED) {
                const double y = (double)x;
                s += y;
                s2 = fma(y, y, s2);
                sj = fma((double)j, y, sj);
            }
        };

        if constexpr (MODE == SLAB_X2X1X1X2 || MODE == SLAB_X2X1) {
            // x2 on the columns (x1 = col_t) of this thread's slab, in LDS
            int sigma;
            const auto kc = axis_coef<T>(job, 1, ik[1], sigma);
            T* col = lds + slab_t * N * PX + col_t;
            dispatch_sigma(sigma, [&](auto sc) {
                T v[N];
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = col[i * PX];
                advect_line<T, N, M, G, CL, decltype(sc)::value>(v, kc, sigma, [&](int j, T x) { col[j * PX] = x; });
            });
            __syncthreads();
        }
        {   // x1 on the rows (x2, slab) = (col_t, slab_t), once or (SLAB_X2X1X1X2) twice.
            // No other thread touches this thread's LDS row, so the two x1 sweeps of
            // SLAB_X2X1X1X2 need no barrier between them.  X1REG (FP32, N <= 64): the
            // intermediate line stays in registers as in k_pencil's two-sweep form (the
            // first sweep's cells for other shifts through the compile-time barrel
            // shifter), which saves a store and a load of the row per lane; the step's
            // partials are tallied from those registers in ascending x1, the order of
            // the LDS form.  Otherwise (FP64 lines) the two sweeps run through the LDS
            // row as a loop kept rolled, so no two lines are live at once.
            int sigma;
            const auto kc = axis_coef<T>(job, 0, ik[0], sigma);
            T* row = lds + threadIdx.x * PX;
            constexpr bool X1REG = MODE == SLAB_X2X1X1X2 && sizeof(T) == 4 && N <= 64;
            if constexpr (X1REG) {
                dispatch_sigma(sigma, [&](auto sc) {
                    constexpr int SIG = decltype(sc)::value;
                    T v[N], y[N];
#pragma unroll
                    for (int i = 0; i < N; ++i) v[i] = row[i];
                    if constexpr (SIG != SIG_ANY) {
                        advect_line<T, N, M, G, CL, SIG>(v, kc, sigma, [&](int j, T x) { y[j] = x; });
                    } else {
                        T cv[N + 7];
                        line_cells<T, N, M, G, CL>(v, cv, kc);
                        store_cells<T, N, SIG_ANY>(cv, sigma, [&](int j, T x) { y[j] = x; });
                    }
                    if constexpr (RED) {   // the step ends after the first x1 sweep
#pragma unroll
                        for (int i = 0; i < N; ++i) tally(i, y[i]);
                    }
                    advect_line<T, N, M, G, CL, SIG>(y, kc, sigma, [&](int j, T x) { row[j] = x; });
                });
            } else {
                constexpr int NX1 = MODE == SLAB_X2X1X1X2 ? 2 : 1;
#pragma unroll 1
                for (int pass = 0; pass < NX1; ++pass) {
                    dispatch_sigma(sigma, [&](auto sc) {
                        T v[N];
#pragma unroll
                        for (int i = 0; i < N; ++i) v[i] = row[i];
                        advect_line<T, N, M, G, CL, decltype(sc)::value>(v, kc, sigma, [&](int j, T x) { row[j] = x; });
                    });
                    if constexpr (RED) {
                        if (pass == 0) {   // the step ends after the first x1 sweep
#pragma unroll
                            for (int i = 0; i < N; ++i) tally(i, row[i]);
                        }
                    }
                }
            }
        }
        __syncthreads();

        if constexpr (MODE == SLAB_X1 || MODE == SLAB_X2X1) {
            const Buf ob(out_ptr, UNIT_BYTES);
            static_for<0, RV>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const int e = q * NT + threadIdx.x;
                const int row = (e * VW) / N, x1 = (e * VW) % N;
                V x;
#pragma unroll
                for (int i = 0; i < VW; ++i) vset<T>(x, i, lds[row * PX + x1 + i]);
                ob.template store16<T, CP>(x, threadIdx.x * 16u, (uint32_t)(q * NT * 16));
            });
        } else {
            // x2 on the columns, stored straight to global memory
            int sigma;
            const auto kc = axis_coef<T>(job, 1, ik[1], sigma);
            const int base = slab_t * N * PX + col_t;
            const Buf ob(out_ptr, UNIT_BYTES);
            const uint32_t voff = (uint32_t)((slab_t * N * N + col_t) * sizeof(T));
            dispatch_sigma(sigma, [&](auto sc) {
                T v[N];
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = lds[base + i * PX];
                advect_line<T, N, M, G, CL, decltype(sc)::value>(
                    v, kc, sigma, [&](int j, T x) { ob.template store<T, CP>(x, voff, (uint32_t)(j * N * sizeof(T))); });
            });
        }
        if constexpr (RED) {
            // this thread's row: x2 = col_t, x3 = slab0 + slab_t; sj carries the x1 index
            double acc[5] = {s, s2, sj, (double)col_t * s, (double)(slab0 + slab_t) * s};
            write_partials<NT>(acc, ik, partials + u * NRED);
        }
        if (next >= units) break;
        __syncthreads();   // the output phase has read the LDS before the next fill
        u = next;
    }
}

// ---------------------------------------------------------------------------
// One line per lane along axis AXIS (1: x2, 2: x3), NT lines per block; NT divides
// N*N so a block never straddles two items.  NSW sweeps along the axis (2: the x3
// sweep that ends one step and the x3 sweep that starts the next, see SlabMode).
// RED: FP64 partials of the field after the first sweep, one row per block.
// OBS (one x3 sweep): partials is the item rows of the observables instead; each lane
// holds its (x1, x2) column after the sweep, so it forms the column sum q and, with
// the other lanes of its wave (64 consecutive columns), the group plane sums G in the
// order of chasm_obs.hpp.
template <typename T, int N, int M, int G, int CL, int NT, int AXIS, int NSW, bool RED, bool OBS = false>
__global__ __launch_bounds__(NT) void k_pencil(const Work w, double* __restrict__ partials)
{
    static_assert((N * N) % NT == 0, "block must tile the lines of one item");
    static_assert(NSW == 1 || NSW == 2, "one or two sweeps");
    constexpr int BPI = N * N / NT;
    long long item;
    const JobDev& job = job_of(w, blockIdx.x / BPI, item);
    const int L = (blockIdx.x % BPI) * NT + threadIdx.x;
    int ik[3];
    item_k(job, item, ik);
    const long long off = item * (long long)(N * N * N);

    // o1, o2: indices of the two other axes (x1 and x2 for AXIS 2, x1 and x3 for AXIS 1)
    const int o1 = L % N, o2 = L / N;
    const int base = AXIS == 2 ? L : o2 * N * N + o1;

    int sigma;
    const auto kc = axis_coef<T>(job, AXIS, ik[AXIS], sigma);
    const Buf buf(static_cast<const T*>(job.f) + off, (uint32_t)(N * N * N * sizeof(T)));
    const Buf obuf(static_cast<T*>(job.out) + off, (uint32_t)(N * N * N * sizeof(T)));
    const uint32_t voff = (uint32_t)base * sizeof(T);
    constexpr uint32_t sstride = (uint32_t)((AXIS == 2 ? N * N : N) * sizeof(T));
    T v[N];
    static_for<0, N>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        v[i] = buf.load<T>(voff, i * sstride);
    });
    if constexpr (OBS) {
        static_assert(AXIS == 2 && NSW == 1 && !RED, "observables in the single x3 sweep");
        T y[N];
        dispatch_sigma(sigma, [&](auto sc) {
            constexpr int SIG = decltype(sc)::value;
            if constexpr (SIG != SIG_ANY) {
                advect_line<T, N, M, G, CL, SIG>(v, kc, sigma, [&](int j, T x) { y[j] = x; });
            } else {
                T cv[N + 7];
                line_cells<T, N, M, G, CL>(v, cv, kc);
                store_cells<T, N, SIG_ANY>(cv, sigma, [&](int j, T x) { y[j] = x; });
            }
        });
        double* const row = partials + item * obs_row(N, N, N);
        double q = 0.0;
        static_for<0, N>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            obuf.store<T>(y[j], voff, j * sstride);
            const double x = (double)y[j];
            q += x;
            const double gs = obs_wave_sum(x);
            if ((threadIdx.x & 63) == 0) row[N * N + (L >> 6) * N + j] = gs;
        });
        row[L] = q;
        return;
    }
    double s = 0.0, s2 = 0.0, sj = 0.0;
    auto tally = [&](int j, T x) {
        if constexpr (RED) {
            const double y = (double)x;
            s += y;
            s2 = fma(y, y, s2);
            sj = fma((double)j, y, sj);
        }
    };
    auto store = [&](int j, T x) { obuf.store<T>(x, voff, j * sstride); };
    dispatch_sigma(sigma, [&](auto sc) {
        constexpr int SIG = decltype(sc)::value;
        if constexpr (NSW == 1) {
            advect_line<T, N, M, G, CL, SIG>(v, kc, sigma, [&](int j, T x) {
                store(j, x);
                tally(j, x);
            });
        } else {
            // The intermediate line stays in this lane's registers.  For SIG_ANY the
            // first sweep's cell values go through the compile-time barrel shifter of
            // store_cells, so no register array is ever indexed at run time (an FP32
            // form that wrote y[j] at the runtime index j compiled to GPR-indexing mode
            // and gave wrong values for those lines on gfx950; its FP64 twin did not).
            T y[N];
            if constexpr (SIG != SIG_ANY) {
                advect_line<T, N, M, G, CL, SIG>(v, kc, sigma, [&](int j, T x) {
                    y[j] = x;
                    tally(j, x);
                });
            } else {
                T cv[N + 7];
                line_cells<T, N, M, G, CL>(v, cv, kc);
                store_cells<T, N, SIG_ANY>(cv, sigma, [&](int j, T x) {
                    y[j] = x;
                    tally(j, x);
                });
            }
            advect_line<T, N, M, G, CL, SIG>(y, kc, sigma, store);
        }
    });
    if constexpr (RED) {
        double acc[5];
        acc[0] = s;
        acc[1] = s2;
        acc[2] = (double)o1 * s;
        if (AXIS == 2) { acc[3] = (double)o2 * s; acc[4] = sj; }
        else { acc[3] = sj; acc[4] = (double)o2 * s; }
        write_partials<NT>(acc, ik, partials + (long long)blockIdx.x * NRED);
    }
}

// ---------------------------------------------------------------------------
// Diagnostics of the current field, one item per block.
template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_reduce_field(const Work w, double* __restrict__ partials)
{
    constexpr int VW = Vec16<T>::n;
    using V = typename Vec16<T>::type;
    long long item;
    const JobDev& job = job_of(w, blockIdx.x, item);
    int ik[3];
    item_k(job, item, ik);
    const V* __restrict__ src = reinterpret_cast<const V*>(static_cast<const T*>(job.f) + item * (long long)(N * N * N));
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = threadIdx.x; e < N * N * N / VW; e += NT) {
        const V x = src[e];
        const int row = (e * VW) / N, x1 = (e * VW) % N;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < VW; ++i) {
            const double y = (double)vget<T>(x, i);
            s += y;
            acc[1] = fma(y, y, acc[1]);
            acc[2] = fma((double)(x1 + i), y, acc[2]);
        }
        acc[0] += s;
        acc[3] = fma((double)(row % N), s, acc[3]);
        acc[4] = fma((double)(row / N), s, acc[4]);
    }
    write_partials<NT>(acc, ik, partials + (long long)blockIdx.x * NRED);
}

struct FinalizeArgs {
    double xlo[3], hx[3], klo[3], hk[3];
    double vol;
};

// Sum the partials of each batch member in a fixed order and convert index moments
// to physical ones.  Block b handles batch member b: partial rows
// [b*rows_per_batch, (b+1)*rows_per_batch).  Results go to out[b*8 .. b*8+7]; when
// hist is non-null they are also appended at history slot *counter (incremented by
// block 0 after all blocks have read it -- one launch, so the read happens first).
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, long long rows_per_batch,
                                                  FinalizeArgs a, double* __restrict__ out,
                                                  double* __restrict__ hist, int* __restrict__ counter,
                                                  int hist_cap, int nbatch);

}  // namespace chasm

// chasm_rt.hip -- runtime-shape kernels of the characteristic step (see chasm_rt.hpp).
//
// One launch per axis sweep.  A block of 64 threads takes L <= 64 lines of one item
// along the sweep axis into LDS (tile [node][line], rows padded to L+1 so every access
// of a wave is bank-conflict free), each thread then runs one line:
//   1. interface slopes (times h) d_q = bias_q + sum_t S[q][t] v(I_q - G + t), the PMBC
//      rows of eqs. 3.4-3.5 truncated to |j - I_q| <= g (clipped to the line);
//   2. per patch the reduced tridiagonal system of the (m+3)-unknown Hermite system of
//      Sec. 3.1.2 step (5), forward and back substitution with the FP64 factors of the
//      host (eta_{-1}, eta_{m+1} from the slope rows);
//   3. the 4-tap cell values of the patch (eqs. 3.7-3.8), written to output node
//      j = c - sigma (the upwind patch evaluates the departure points in its cells,
//      correction procedure of Sec. 3.1.3), outer ghosts as in the compiled kernels;
// and the tile goes back to HBM with the same coalesced traversal.  The arithmetic of a
// line is the same, operation for operation, as the compiled line routine
// (chasm_line.hpp), with the tables read at run time.
#include "chasm_rt.hpp"

#include "chasm_kernels.hpp"

namespace chasm {

constexpr int kRtThreads = 64;
constexpr size_t kRtLds = 64 * 1024;

static size_t rt_tile_elems(const RtAxis& a, int L)
{
    return (size_t)(2 * a.N + a.M + 3 + a.P + 1) * (size_t)(L + 1);
}

int rt_lines_per_block(const RtJob& j, int axis, int elem_bytes)
{
    for (int L = 64; L >= 16; L /= 2)
        if (rt_tile_elems(j.ax[axis], L) * (size_t)elem_bytes <= kRtLds) return L;
    return 0;
}

static int rt_lines(const RtJob& j, int axis)
{
    return j.nx[0] * j.nx[1] * j.nx[2] / j.nx[axis];
}

long long rt_rows_per_item(const RtJob& j, int dtype)
{
    const int L = rt_lines_per_block(j, 2, dtype == 1 ? 8 : 4);
    return L ? (rt_lines(j, 2) + L - 1) / L : 0;
}

__device__ __forceinline__ void rt_item_k(const RtJob& j, long long item, int ik[3])
{
    const long long nkp = (long long)j.nk[0] * j.nk[1] * j.nk[2];
    const long long kf = item % nkp;
    ik[0] = (int)(kf % j.nk[0]);
    ik[1] = (int)((kf / j.nk[0]) % j.nk[1]);
    ik[2] = (int)(kf / ((long long)j.nk[0] * j.nk[1]));
}

template <typename T, int AXIS, bool RED>
__global__ __launch_bounds__(kRtThreads) void k_rt_sweep(const RtJob j, int L, double* __restrict__ partials)
{
    extern __shared__ __align__(16) unsigned char rt_smem[];
    T* const sm = reinterpret_cast<T*>(rt_smem);
    const RtAxis& A = j.ax[AXIS];
    const int N = A.N, M = A.M, P = A.P, G = A.G, W = 2 * G + 1;
    const int n0 = j.nx[0], n1 = j.nx[1], n2 = j.nx[2];
    const long long cube = (long long)n0 * n1 * n2;
    const int nlines = (int)(cube / N);
    const int bpi = (nlines + L - 1) / L;
    const long long item = blockIdx.x / bpi;
    const int line0 = (int)(blockIdx.x % bpi) * L;
    const int nl = min(L, nlines - line0);
    const int LP = L + 1;
    T* const tin = sm;
    T* const tout = tin + N * LP;
    T* const eb = tout + N * LP;
    T* const db = eb + (M + 3) * LP;
    const T* const src = static_cast<const T*>(j.f) + item * cube;
    T* const dst = static_cast<T*>(j.out) + item * cube;
    const int tid = threadIdx.x;
    const long long stride = AXIS == 0 ? 1 : (AXIS == 1 ? (long long)n0 : (long long)n0 * n1);
    // first element of this thread's line (lines along x1: rows; x2: (x1, x3); x3: (x1, x2))
    const int lg = line0 + tid;
    const long long lbase = AXIS == 0 ? (long long)lg * n0
                                      : (AXIS == 1 ? (long long)(lg / n0) * n0 * n1 + lg % n0 : (long long)lg);

    if (AXIS == 0) {            // rows are contiguous: lanes along the row
        for (int r = 0; r < nl; ++r)
            for (int i = tid; i < N; i += kRtThreads) tin[i * LP + r] = src[(long long)(line0 + r) * n0 + i];
    } else if (tid < nl) {      // lanes along x1: every load of the wave is a run of x1
        for (int i = 0; i < N; ++i) tin[i * LP + tid] = src[lbase + i * stride];
    }
    __syncthreads();

    int ik[3];
    rt_item_k(j, item, ik);
    const int sigma = ((const int __attribute__((address_space(4)))*)A.shift)[ik[AXIS]];
    const cptr<T> wk = (cptr<T>)(A.w) + 4 * ik[AXIS];
    const T w0 = wk[0], w1 = wk[1], w2 = wk[2], w3 = wk[3];
    double s = 0.0, s2 = 0.0, sj = 0.0;
    if (tid < nl) {
        const T* const v = tin + tid;
        T* const o = tout + tid;
        T* const e = eb + tid;
        T* const d = db + tid;
        const cptr<T> st = (cptr<T>)A.stencil;
        const cptr<T> bi = (cptr<T>)A.bias;
        // 1. interface slopes times h
        for (int q = 0; q <= P; ++q) {
            const int I = q < P ? q * M : N - 1;
            const int j0 = I - G < 0 ? 0 : I - G, j1 = I + G > N - 1 ? N - 1 : I + G;
            T acc = bi[q];
            for (int jj = j0; jj <= j1; ++jj) acc = fma(st[q * W + (jj - I + G)], v[jj * LP], acc);
            d[q * LP] = acc;
        }
        // 2.-3. patches: eta_{u-1} at e[u], u = 0 .. m+2
        for (int l = 0; l < P; ++l) {
            const int s0 = l * M, m = l == P - 1 ? A.MLAST : M;
            const cptr<T> f3 = (cptr<T>)(A.lu) + (m == M ? 0 : 3 * (M + 1));
            const cptr<T> inv = f3, ainv = f3 + (M + 1), cpv = f3 + 2 * (M + 1);
            const T dl = d[l * LP], dr = d[(l + 1) * LP];
            T prev = fma(T(1.0 / 3.0), dl, v[s0 * LP]) * inv[0];
            e[LP] = prev;
            for (int i = 1; i <= m; ++i) {
                T r = v[(s0 + i) * LP];
                if (i == m) r = fma(T(-1.0 / 3.0), dr, r);
                prev = fma(-ainv[i], prev, r * inv[i]);
                e[(i + 1) * LP] = prev;
            }
            T nxt = prev;
            for (int i = m - 1; i >= 0; --i) {
                nxt = fma(-cpv[i], nxt, e[(i + 1) * LP]);
                e[(i + 1) * LP] = nxt;
            }
            e[0] = fma(T(-2), dl, e[2 * LP]);
            e[(m + 2) * LP] = fma(T(2), dr, e[m * LP]);
            auto put = [&](int c, T x) {
                const int jo = c - sigma;
                if (jo >= 0 && jo < N) o[jo * LP] = x;
            };
            for (int nu = 0; nu < m; ++nu) {
                T a = w0 * e[nu * LP];
                a = fma(w1, e[(nu + 1) * LP], a);
                a = fma(w2, e[(nu + 2) * LP], a);
                a = fma(w3, e[(nu + 3) * LP], a);
                put(s0 + nu, a);
            }
            if (l == 0) {
                const T e0 = e[0], e1 = e[LP], e2 = e[2 * LP], e3 = e[3 * LP];
                const T gl = A.poly3 ? (4 * e0 - 6 * e1 + 4 * e2 - e3) : T(0);
                put(-1, fma(w3, e2, fma(w2, e1, fma(w1, e0, w0 * gl))));
                put(-2, fma(w3, e1, fma(w2, e0, w1 * gl)));
                put(-3, fma(w3, e0, w2 * gl));
                put(-4, w3 * gl);
            }
            if (l == P - 1) {
                const T em1 = e[(m - 1) * LP], em = e[m * LP], ep1 = e[(m + 1) * LP], ep2 = e[(m + 2) * LP];
                const T gr = A.poly3 ? (4 * ep2 - 6 * ep1 + 4 * em - em1) : T(0);
                put(N - 1, fma(w3, gr, fma(w2, ep2, fma(w1, ep1, w0 * em))));
                put(N, fma(w2, gr, fma(w1, ep2, w0 * ep1)));
                put(N + 1, fma(w1, gr, w0 * ep2));
                put(N + 2, w0 * gr);
            }
        }
        // output nodes whose departure cell lies beyond the ghost cells
        for (int jo = 0; jo < N; ++jo) {
            const int c = jo + sigma;
            if (c < -4 || c > N + 2) o[jo * LP] = T(0);
        }
        if constexpr (RED) {
            for (int jo = 0; jo < N; ++jo) {
                const double y = (double)o[jo * LP];
                s += y;
                s2 = fma(y, y, s2);
                sj = fma((double)jo, y, sj);
            }
        }
    }
    __syncthreads();

    if (AXIS == 0) {
        for (int r = 0; r < nl; ++r)
            for (int i = tid; i < N; i += kRtThreads) dst[(long long)(line0 + r) * n0 + i] = tout[i * LP + r];
    } else if (tid < nl) {
        for (int i = 0; i < N; ++i) dst[lbase + i * stride] = tout[i * LP + tid];
    }
    if constexpr (RED) {
        static_assert(AXIS == 2, "the step ends with the x3 sweep");
        double acc[5] = {s, s2, (double)(lg % n0) * s, (double)(lg / n0) * s, sj};
        if (tid >= nl) acc[0] = acc[1] = acc[2] = acc[3] = acc[4] = 0.0;
        write_partials<kRtThreads>(acc, ik, partials + (long long)blockIdx.x * NRED);
    }
}

template <typename T>
static hipError_t rt_sweep_t(const RtJob& j, int axis, double* partials, hipStream_t s)
{
    const int L = rt_lines_per_block(j, axis, sizeof(T));
    if (L == 0) return hipErrorInvalidConfiguration;
    const long long bpi = (rt_lines(j, axis) + L - 1) / L;
    const unsigned grid = (unsigned)(j.nitems * bpi);
    const size_t lds = rt_tile_elems(j.ax[axis], L) * sizeof(T);
    switch (axis) {
    case 0: hipLaunchKernelGGL((k_rt_sweep<T, 0, false>), dim3(grid), dim3(kRtThreads), lds, s, j, L, partials); break;
    case 1: hipLaunchKernelGGL((k_rt_sweep<T, 1, false>), dim3(grid), dim3(kRtThreads), lds, s, j, L, partials); break;
    default:
        if (partials)
            hipLaunchKernelGGL((k_rt_sweep<T, 2, true>), dim3(grid), dim3(kRtThreads), lds, s, j, L, partials);
        else
            hipLaunchKernelGGL((k_rt_sweep<T, 2, false>), dim3(grid), dim3(kRtThreads), lds, s, j, L, partials);
        break;
    }
    return hipGetLastError();
}

hipError_t rt_sweep(const RtJob& j, int axis, int dtype, double* partials, hipStream_t s)
{
    return dtype == 1 ? rt_sweep_t<double>(j, axis, partials, s) : rt_sweep_t<float>(j, axis, partials, s);
}

// Diagnostics of the current field, one item per block: threads own (x1, x2) columns.
template <typename T>
__global__ __launch_bounds__(256) void k_rt_reduce(const RtJob j, double* __restrict__ partials)
{
    const int n0 = j.nx[0], n1 = j.nx[1], n2 = j.nx[2];
    const long long plane = (long long)n0 * n1;
    const long long item = blockIdx.x;
    const T* src = static_cast<const T*>(j.f) + item * plane * n2;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long p = threadIdx.x; p < plane; p += 256) {
        const int x1 = (int)(p % n0), x2 = (int)(p / n0);
        double c = 0.0, c2 = 0.0, c3 = 0.0;
        for (int x3 = 0; x3 < n2; ++x3) {
            const double y = (double)src[x3 * plane + p];
            c += y;
            c2 = fma(y, y, c2);
            c3 = fma((double)x3, y, c3);
        }
        acc[0] += c;
        acc[1] += c2;
        acc[2] = fma((double)x1, c, acc[2]);
        acc[3] = fma((double)x2, c, acc[3]);
        acc[4] += c3;
    }
    int ik[3];
    rt_item_k(j, item, ik);
    write_partials<256>(acc, ik, partials + item * NRED);
}

hipError_t rt_reduce(const RtJob& j, int dtype, double* partials, hipStream_t s)
{
    const unsigned grid = (unsigned)j.nitems;
    if (dtype == 1)
        hipLaunchKernelGGL((k_rt_reduce<double>), dim3(grid), dim3(256), 0, s, j, partials);
    else
        hipLaunchKernelGGL((k_rt_reduce<float>), dim3(grid), dim3(256), 0, s, j, partials);
    return hipGetLastError();
}

}  // namespace chasm

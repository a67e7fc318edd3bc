// chasm_rt.hip -- runtime-shape kernels of the characteristic step (see chasm_rt.hpp).
//
// One launch per axis sweep.  Every line runs the same arithmetic, operation for
// operation, as the compiled line routine (chasm_line.hpp), with the tables read at run
// time:
//   1. interface slopes (times h) d_q = bias_q + sum_t S[q][t] v(I_q - G + t), the PMBC
//      rows of eqs. 3.4-3.5 truncated to |j - I_q| <= g (clipped to the line);
//   2. per patch the reduced tridiagonal system of the (m+3)-unknown Hermite system of
//      Sec. 3.1.2 step (5), forward and back substitution with the FP64 factors of the
//      host (eta_{-1}, eta_{m+1} from the slope rows);
//   3. the 4-tap cell values of the patch (eqs. 3.7-3.8), written to output node
//      j = c - sigma (the upwind patch evaluates the departure points in its cells,
//      correction procedure of Sec. 3.1.3), outer ghosts as in the compiled kernels.
//
// k_rt_patch (the fast form; patches of up to 64 cells, up to 8 patches a line): a
// block of 64 PW threads takes L <= 64 lines of one item into one LDS tile [node][line]
// (rows padded to 65 so every access of a wave is bank-conflict free) with batched,
// coalesced loads (sixteen in flight per thread); lane = line, wave = patch.  The wave
// index is made explicitly uniform, so a patch's table rows come in as wide scalar
// loads and its branches are scalar; item and k-point arithmetic stays in 32 bits.
// Each thread solves its own patch with the unknowns eta in VGPRs, and after a barrier,
// when every read of the tile is done, writes its cell values into the same tile in
// place: every output node takes exactly one value (from the patch owning its
// departure cell, or zero beyond the ghosts), so the writes never collide.  The tile
// then goes back with the same coalesced traversal.  The paper's lines (n_nb = 15 with
// patches of 10, 15 or 20 cells) have compile-time forms: their loops are unrolled
// without guards and their tile carries zero rows beyond both ends, so each slope is 31
// taps at fixed LDS offsets with the coefficients in SGPRs.  Consecutive blocks are dealt to the XCDs so
// that neighbouring tiles share an L2.
//
// k_rt_sweep (every other shape): one 64-thread block of L <= 64 lines, one line per
// thread, separate LDS input and output tiles and LDS rows for eta and the slopes.
#include "chasm_rt.hpp"

#include "chasm_kernels.hpp"
#include "chasm_obs.hpp"

namespace chasm {

constexpr int kRtThreads = 64;
constexpr size_t kRtLds = 64 * 1024;
constexpr int kRpLines = 64;        // lines per block of k_rt_patch (lane = line)
constexpr int kRpMaxPatches = 8;    // waves per block of k_rt_patch (wave = patch)

static size_t rt_tile_elems(const RtAxis& a, int L)
{
    return (size_t)(2 * a.N + a.M + 3 + a.P + 1) * (size_t)(L + 1);
}

// Waves per block of k_rt_patch for this axis (the least power of two >= P), or 0 when
// the line does not fit its form: patches of more than 64 cells, more than 8 patches,
// or a tile of more than 63 KB (the block's partial sums take the rest).
static int rp_tile_rows(const RtAxis& a);

static int rp_waves(const RtAxis& a, int elem_bytes)
{
    if (a.M > 64 || a.P > kRpMaxPatches) return 0;
    if ((size_t)rp_tile_rows(a) * (kRpLines + 1) * (size_t)elem_bytes > kRtLds - 1024) return 0;
    int pw = 1;
    while (pw < a.P) pw *= 2;
    return pw;
}

// Lines along x2 of k_rt_patch: whole x3-planes (a multiple of n0, so each node's run
// is whole rows) when that fills at least 56 of the 64 lanes; else 64 lines (0 here).
static int rp_plane_lines(const RtJob& j)
{
    const int lines = j.nx[0] <= kRpLines ? (kRpLines / j.nx[0]) * j.nx[0] : 0;
    return lines >= 56 ? lines : 0;
}

int rt_lines_per_block(const RtJob& j, int axis, int elem_bytes)
{
    if (rp_waves(j.ax[axis], elem_bytes)) return axis == 1 && rp_plane_lines(j) ? rp_plane_lines(j) : kRpLines;
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

// k-point of an item (items are < 2^31: the host bounds every launch grid), in 32-bit
// arithmetic: a 64-bit division costs a hundred scalar instructions.
__device__ __forceinline__ void rt_item_k(const RtJob& j, unsigned item, int ik[3])
{
    const unsigned nk0 = (unsigned)j.nk[0], nk1 = (unsigned)j.nk[1];
    const unsigned kf = item % (nk0 * nk1 * (unsigned)j.nk[2]);
    ik[0] = (int)(kf % nk0);
    ik[1] = (int)((kf / nk0) % nk1);
    ik[2] = (int)(kf / (nk0 * nk1));
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

// Workgroups are dealt to the eight XCDs in turn; give XCD x the x-th eighth of the
// logical blocks, so that neighbouring tiles (which share cache lines at their edges)
// meet in the same L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned full = nb & ~7u;
    return b >= full ? b : (b & 7u) * (full >> 3) + (b >> 3);
}

// The last four unknowns of a patch, eta_{m-2} .. eta_{m+1}: the right ghost
// evaluations read them, and the last cell's 4-tap sum reads eta_{m+1}.
template <typename T>
struct RtTail {
    T em1, em, ep1, ep2;
};

// One patch of one line (lane): slopes at its two interfaces, the reduced tridiagonal
// system, eta_{u-1} into e[u] for u = 0 .. m+1 (m == MB: also e[m+2]) and the tail.
// v: the line in the tile (node i at v[i * LP]).  GS > 0: the ghost width is GS and the
// tile carries zero rows beyond both ends of the line, so every slope runs all
// 2 GS + 1 taps with compile-time offsets (a clipped tap adds fma(0, 0, acc) = acc,
// bitwise the clipped sum); GS == 0: runtime width, taps clipped to the line, eight at
// a time.  m == MB: fully unrolled; m < MB: guarded by m, nodes and factors fetched
// sixteen at a time, and the tail captured as the back substitution passes it (no
// register array is ever indexed by m).
template <typename T, int MB, int GS>
__device__ __forceinline__ RtTail<T> rt_solve_patch(const RtAxis& A, const T* v, int l, int m, T (&e)[MB + 3])
{
    constexpr int LP = kRpLines + 1;
    const int N = A.N, M = A.M, P = A.P, G = GS ? GS : A.G, W = 2 * G + 1;
    const int s0 = l * M;
    const cptr<T> st = (cptr<T>)A.stencil;
    const cptr<T> bi = (cptr<T>)A.bias;
    auto slope = [&](int q) {
        const int I = q < P ? q * M : N - 1;
        T acc = bi[q];
        if constexpr (GS > 0) {
            const T* const vw = v + (I - GS) * LP;
            const cptr<T> row = st + q * W;
#pragma unroll
            for (int t = 0; t < 2 * GS + 1; ++t) acc = fma(row[t], vw[t * LP], acc);
        } else {
            const int j0 = I - G < 0 ? 0 : I - G, j1 = I + G > N - 1 ? N - 1 : I + G;
            const int rb = q * W - I + G;              // coefficient of node jj at st[rb + jj]
            for (int c = j0; c <= j1; c += 8) {
                T cf[8], vv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int jj = min(c + u, j1);
                    cf[u] = st[rb + jj];
                    vv[u] = v[jj * LP];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (c + u <= j1) acc = fma(cf[u], vv[u], acc);
            }
        }
        return acc;
    };
    const T dl = slope(l), dr = slope(l + 1);
    const cptr<T> f3 = (cptr<T>)(A.lu) + (m == M ? 0 : 3 * (M + 1));
    const cptr<T> inv = f3, ainv = f3 + (M + 1), cpv = f3 + 2 * (M + 1);
    T prev = fma(T(1.0 / 3.0), dl, v[s0 * LP]) * inv[0];
    e[1] = prev;
    RtTail<T> t;
    if (m == MB) {
#pragma unroll
        for (int i = 1; i <= MB; ++i) {
            T r = v[(s0 + i) * LP];
            if (i == MB) r = fma(T(-1.0 / 3.0), dr, r);
            prev = fma(-ainv[i], prev, r * inv[i]);
            e[i + 1] = prev;
        }
        T nxt = prev;
#pragma unroll
        for (int i = MB - 1; i >= 0; --i) {
            nxt = fma(-cpv[i], nxt, e[i + 1]);
            e[i + 1] = nxt;
        }
        e[0] = fma(T(-2), dl, e[2]);
        e[MB + 2] = fma(T(2), dr, e[MB]);
        t.em1 = e[MB - 1];
        t.em = e[MB];
        t.ep1 = e[MB + 1];
        t.ep2 = e[MB + 2];
        return t;
    }
#pragma unroll
    for (int c = 0; c < MB; c += 16) {
        if (c + 1 <= m) {
            T vv[16], iv[16], ai[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = min(c + 1 + u, m);
                vv[u] = v[(s0 + i) * LP];
                iv[u] = inv[i];
                ai[u] = ainv[i];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int i = c + 1 + u;
                if (i > MB) break;                      // compile-time: the array holds MB + 3
                if (i <= m) {
                    T r = vv[u];
                    if (i == m) r = fma(T(-1.0 / 3.0), dr, r);
                    prev = fma(-ai[u], prev, r * iv[u]);
                    e[i + 1] = prev;
                }
            }
        }
    }
    t.ep1 = prev;                                       // eta_m
    T nxt = prev, em = prev, em1 = prev;
#pragma unroll
    for (int c = ((MB - 1) / 16) * 16; c >= 0; c -= 16) {
        if (c <= m - 1) {
            T cp[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) cp[u] = cpv[min(c + u, m - 1)];
#pragma unroll
            for (int u = 15; u >= 0; --u) {
                const int i = c + u;
                if (i > MB - 1) continue;               // compile-time, as above
                if (i <= m - 1) {
                    nxt = fma(-cp[u], nxt, e[i + 1]);
                    e[i + 1] = nxt;
                    if (i == m - 1) em = nxt;           // eta_{m-1}
                    if (i == m - 2) em1 = nxt;          // eta_{m-2}
                }
            }
        }
    }
    e[0] = fma(T(-2), dl, e[2]);
    t.em = em;
    t.em1 = m >= 2 ? em1 : e[0];
    t.ep2 = fma(T(2), dr, em);                          // eta_{m+1}
    return t;
}

// Zero rows of the padded tile of k_rt_patch with GS > 0: the departure cells of the
// ghost evaluations (up to 4 beyond the line) shifted by |sigma| <= GS land in them.
template <int GS>
constexpr int rt_pad() { return GS > 0 ? GS + 4 : 0; }

// The fast form (see the head of this file).  Block: L <= 64 lines of one item, PW
// waves; MB >= M bounds the patch length of the register arrays (MB == M: unrolled).
// Lines along x1 are rows, and the block's values one contiguous run moved as flat
// coalesced runs; along x2 and x3, lane = line for the loads and stores (along x2, L is
// a multiple of n0 when that fills at least 56 lanes, so each node's run is whole rows).
// OBS (x3 sweep, L = 64): partials is the item rows of the observables; the block's 64
// lines are one 64-column group of chasm_obs.hpp, so after the sweep its waves form
// that group's plane sums G and the first wave the column sums q, from the tile.
template <typename T, int AXIS, bool RED, int MB, int PW, int GS, bool OBS = false>
__global__ __launch_bounds__(64 * PW) void k_rt_patch(const RtJob j, int L, double* __restrict__ partials)
{
    constexpr int NT = 64 * PW, LP = kRpLines + 1, PAD = rt_pad<GS>();
    constexpr int U = 16;                       // loads (stores) in flight per thread and round
    extern __shared__ __align__(16) unsigned char rt_smem[];
    T* const tile = reinterpret_cast<T*>(rt_smem) + PAD * LP;   // node i of line r at tile[i * LP + r]
    const RtAxis& A = j.ax[AXIS];
    const int N = A.N;
    const int n0 = j.nx[0], n1 = j.nx[1], n2 = j.nx[2];
    const long long cube = (long long)n0 * n1 * n2;
    const int nlines = n0 * n1 * n2 / N;
    const unsigned bpi = (unsigned)((nlines + L - 1) / L);
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const unsigned item = blk / bpi;
    const int line0 = (int)(blk % bpi) * L;
    const int nl = min(L, nlines - line0);
    const T* const src = static_cast<const T*>(j.f) + (long long)item * cube;
    T* const dst = static_cast<T*>(j.out) + (long long)item * cube;
    // the wave index is uniform over the wave: say so, so that the patch, its table rows
    // and its branches live in SGPRs (scalar loads, no exec masking)
    const int tid = threadIdx.x, ln = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    // lane = line: consecutive lanes are consecutive x1 (lines along x2: (x1, x3); x3: (x1, x2))
    const int lg = line0 + ln;
    const long long lbase = AXIS == 1 ? (long long)(lg / n0) * n0 * n1 + lg % n0 : (long long)lg;
    const long long stride = AXIS == 1 ? (long long)n0 : (long long)n0 * n1;
    const long long fbase = (long long)line0 * N;
    const int cnt = nl * N;

    // row of element idx of the run: idx < 64 N <= 2^14 and N <= 256, so the FP32
    // quotient (idx + 1/2) / N is never within 1/(2N) of an integer and its error is
    // below 2^-16: truncation gives floor(idx / N) exactly, without an integer division
    const float rN = 1.0f / (float)N;
    auto row_of = [&](int idx) { return (int)(((float)idx + 0.5f) * rN); };
    if (AXIS == 0) {
        for (int i0 = tid; i0 < cnt; i0 += U * NT) {
            T x[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * NT < cnt) x[u] = src[fbase + i0 + u * NT];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = i0 + u * NT;
                if (idx < cnt) {
                    const int r = row_of(idx);
                    tile[(idx - r * N) * LP + r] = x[u];
                }
            }
        }
    } else if (ln < nl) {
        for (int i0 = wv; i0 < N; i0 += U * PW) {
            T x[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * PW < N) x[u] = src[lbase + (long long)(i0 + u * PW) * stride];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * PW < N) tile[(i0 + u * PW) * LP + ln] = x[u];
        }
    }
    if constexpr (PAD > 0) {
        for (int idx = tid; idx < 2 * PAD * 64; idx += NT) {
            const int row = idx >> 6;
            tile[(row < PAD ? row - PAD : N + row - PAD) * LP + (idx & 63)] = T(0);
        }
    }
    __syncthreads();

    int ik[3];
    rt_item_k(j, item, ik);
    const int sigma = ((const int __attribute__((address_space(4)))*)A.shift)[ik[AXIS]];
    const cptr<T> wk = (cptr<T>)(A.w) + 4 * ik[AXIS];
    const T w0 = wk[0], w1 = wk[1], w2 = wk[2], w3 = wk[3];
    const int M = A.M, P = A.P;
    const int l = wv;                                   // this wave's patch
    const int s0 = l * M, m = l == P - 1 ? A.MLAST : M;
    T* const v = tile + ln;                             // this lane's line, node i at v[i * LP]
    T e[MB + 3];                                        // eta_{u-1} at e[u]
#pragma unroll
    for (int u = 0; u < MB + 3; ++u) e[u] = T(0);
    RtTail<T> tl{T(0), T(0), T(0), T(0)};
    if (l < P) tl = rt_solve_patch<T, MB, GS>(A, v, l, m, e);
    __syncthreads();    // every read of the tile is done: the values go back in place

    if (l < P) {
        // 3. cell values of the patch, then its outer ghosts; with the padded tile and
        //    |sigma| <= GS every target row exists and the rows beyond the line are
        //    never stored, so the writes need no test
        const bool open = PAD > 0 && sigma >= -GS && sigma <= GS;
        auto put = [&](int c, T x) {
            const int jo = c - sigma;
            if (open || (jo >= 0 && jo < N)) v[jo * LP] = x;
        };
        if (m == MB) {
#pragma unroll
            for (int nu = 0; nu < MB; ++nu) {
                T a = w0 * e[nu];
                a = fma(w1, e[nu + 1], a);
                a = fma(w2, e[nu + 2], a);
                a = fma(w3, e[nu + 3], a);
                put(s0 + nu, a);
            }
        } else {
#pragma unroll
            for (int nu = 0; nu < MB; ++nu) {
                if (nu < m) {
                    T a = w0 * e[nu];
                    a = fma(w1, e[nu + 1], a);
                    a = fma(w2, e[nu + 2], a);
                    a = fma(w3, nu == m - 1 ? tl.ep2 : e[nu + 3], a);
                    put(s0 + nu, a);
                }
            }
        }
        if (l == 0) {
            const T e0 = e[0], e1 = e[1], e2 = e[2], e3 = m == 1 ? tl.ep2 : e[3];
            const T gl = A.poly3 ? (4 * e0 - 6 * e1 + 4 * e2 - e3) : T(0);
            put(-1, fma(w3, e2, fma(w2, e1, fma(w1, e0, w0 * gl))));
            put(-2, fma(w3, e1, fma(w2, e0, w1 * gl)));
            put(-3, fma(w3, e0, w2 * gl));
            put(-4, w3 * gl);
        }
        if (l == P - 1) {
            const T em1 = tl.em1, em = tl.em, ep1 = tl.ep1, ep2 = tl.ep2;
            const T gr = A.poly3 ? (4 * ep2 - 6 * ep1 + 4 * em - em1) : T(0);
            put(N - 1, fma(w3, gr, fma(w2, ep2, fma(w1, ep1, w0 * em))));
            put(N, fma(w2, gr, fma(w1, ep2, w0 * ep1)));
            put(N + 1, fma(w1, gr, w0 * ep2));
            put(N + 2, w0 * gr);
        }
    }
    // output nodes whose departure cell lies beyond the ghost cells (no patch writes them)
    if (sigma < -4 || sigma > 3) {
        for (int jo = wv; jo < N; jo += PW) {
            const int c = jo + sigma;
            if (c < -4 || c > N + 2) v[jo * LP] = T(0);
        }
    }
    __syncthreads();

    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (AXIS == 0) {
        for (int i0 = tid; i0 < cnt; i0 += U * NT) {
            T x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = i0 + u * NT;
                if (idx < cnt) {
                    const int r = row_of(idx);
                    x[u] = tile[(idx - r * N) * LP + r];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * NT < cnt) dst[fbase + i0 + u * NT] = x[u];
        }
    } else if (ln < nl) {
        for (int i0 = wv; i0 < N; i0 += U * PW) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * PW;
                if (i < N) {
                    const T y = tile[i * LP + ln];
                    dst[lbase + (long long)i * stride] = y;
                    if constexpr (RED) {
                        const double yd = (double)y;
                        acc[0] += yd;
                        acc[1] = fma(yd, yd, acc[1]);
                        acc[4] = fma((double)i, yd, acc[4]);
                    }
                }
            }
        }
    }
    if constexpr (RED) {
        static_assert(AXIS == 2, "the step ends with the x3 sweep");
        acc[2] = (double)(lg % n0) * acc[0];
        acc[3] = (double)(lg / n0) * acc[0];
        write_partials<NT>(acc, ik, partials + (long long)blk * NRED);
    }
    if constexpr (OBS) {
        static_assert(AXIS == 2 && !RED, "observables in the x3 sweep");
        double* const row = partials + (long long)item * obs_row(n0, n1, N);
        const long long grp = line0 >> 6;
        const bool in = ln < nl;
        for (int z = wv; z < N; z += PW) {
            const double x = in ? (double)tile[z * LP + ln] : 0.0;
            const double gs = obs_wave_sum(x);
            if (ln == 0) row[(long long)n0 * n1 + grp * N + z] = gs;
        }
        if (wv == 0 && in) {
            double q = 0.0;
            for (int z = 0; z < N; ++z) q += (double)tile[z * LP + ln];
            row[lg] = q;
        }
    }
}

template <typename T, int AXIS, bool RED, int MB, int GS, bool OBS>
static void launch_rp(int pw, unsigned grid, size_t lds, hipStream_t s, const RtJob& j, int L, double* partials)
{
    switch (pw) {
    case 1:
        hipLaunchKernelGGL((k_rt_patch<T, AXIS, RED, MB, 1, GS, OBS>), dim3(grid), dim3(64), lds, s, j, L, partials);
        break;
    case 2:
        hipLaunchKernelGGL((k_rt_patch<T, AXIS, RED, MB, 2, GS, OBS>), dim3(grid), dim3(128), lds, s, j, L, partials);
        break;
    case 4:
        hipLaunchKernelGGL((k_rt_patch<T, AXIS, RED, MB, 4, GS, OBS>), dim3(grid), dim3(256), lds, s, j, L, partials);
        break;
    default:
        hipLaunchKernelGGL((k_rt_patch<T, AXIS, RED, MB, 8, GS, OBS>), dim3(grid), dim3(512), lds, s, j, L, partials);
        break;
    }
}

// Register bound and fixed ghost width of k_rt_patch for an axis: the paper's lines
// (n_nb = 15 with patches of 10, 15 or 20 cells: the 41-, 61- and 81-node lines of four
// patches) unrolled with a padded tile; otherwise MB = 16 or 64 with runtime ghost width.
static void rp_variant(const RtAxis& a, int& mb, int& gs)
{
    if (a.G == 15 && (a.M == 10 || a.M == 15 || a.M == 20)) {
        mb = a.M;
        gs = 15;
    } else {
        mb = a.M <= 16 ? 16 : 64;
        gs = 0;
    }
}

static int rp_tile_rows(const RtAxis& a)
{
    int mb, gs;
    rp_variant(a, mb, gs);
    return a.N + 2 * (gs > 0 ? gs + 4 : 0);
}

template <typename T, int AXIS, bool RED, bool OBS = false>
static void launch_rp_mb(const RtAxis& a, int pw, unsigned grid, size_t lds, hipStream_t s, const RtJob& j, int L,
                         double* partials)
{
    int mb, gs;
    rp_variant(a, mb, gs);
    if (gs == 15 && mb == 15)
        launch_rp<T, AXIS, RED, 15, 15, OBS>(pw, grid, lds, s, j, L, partials);
    else if (gs == 15 && mb == 20)
        launch_rp<T, AXIS, RED, 20, 15, OBS>(pw, grid, lds, s, j, L, partials);
    else if (gs == 15 && mb == 10)
        launch_rp<T, AXIS, RED, 10, 15, OBS>(pw, grid, lds, s, j, L, partials);
    else if (mb == 16)
        launch_rp<T, AXIS, RED, 16, 0, OBS>(pw, grid, lds, s, j, L, partials);
    else
        launch_rp<T, AXIS, RED, 64, 0, OBS>(pw, grid, lds, s, j, L, partials);
}

template <typename T>
static hipError_t rt_sweep_t(const RtJob& j, int axis, double* partials, hipStream_t s)
{
    const int L = rt_lines_per_block(j, axis, sizeof(T));
    if (L == 0) return hipErrorInvalidConfiguration;
    const long long bpi = (rt_lines(j, axis) + L - 1) / L;
    const unsigned grid = (unsigned)(j.nitems * bpi);
    const int pw = rp_waves(j.ax[axis], sizeof(T));
    if (pw) {
        const RtAxis& a = j.ax[axis];
        const size_t lds = (size_t)rp_tile_rows(a) * (kRpLines + 1) * sizeof(T);
        switch (axis) {
        case 0: launch_rp_mb<T, 0, false>(a, pw, grid, lds, s, j, L, partials); break;
        case 1: launch_rp_mb<T, 1, false>(a, pw, grid, lds, s, j, L, partials); break;
        default:
            if (partials)
                launch_rp_mb<T, 2, true>(a, pw, grid, lds, s, j, L, partials);
            else
                launch_rp_mb<T, 2, false>(a, pw, grid, lds, s, j, L, partials);
            break;
        }
        return hipGetLastError();
    }
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

bool rt_can_observe(const RtJob& j, int dtype) { return rp_waves(j.ax[2], dtype == 1 ? 8 : 4) != 0; }

template <typename T>
static hipError_t rt_sweep_obs_t(const RtJob& j, double* rows, hipStream_t s)
{
    const RtAxis& a = j.ax[2];
    const int pw = rp_waves(a, sizeof(T));
    if (!pw) return hipErrorNotSupported;
    const int L = kRpLines;
    const unsigned grid = (unsigned)(j.nitems * ((rt_lines(j, 2) + L - 1) / L));
    const size_t lds = (size_t)rp_tile_rows(a) * (kRpLines + 1) * sizeof(T);
    launch_rp_mb<T, 2, false, true>(a, pw, grid, lds, s, j, L, rows);
    return hipGetLastError();
}

hipError_t rt_sweep_obs(const RtJob& j, int dtype, double* rows, hipStream_t s)
{
    return dtype == 1 ? rt_sweep_obs_t<double>(j, rows, s) : rt_sweep_obs_t<float>(j, rows, s);
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

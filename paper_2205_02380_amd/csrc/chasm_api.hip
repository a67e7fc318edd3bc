// chasm_api.hip -- C ABI of the characteristic (spatial-advection) step:
// descriptor validation, FP64 table upload, kernel selection, step scheduling
// (eager or HIP-graph replay), FP64 diagnostics.  See include/chasm_advect.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/chasm_advect.h"
#include "chasm_kernels.hpp"
#include "chasm_registry.hpp"
#include "chasm_rt.hpp"
#include "chasm_tables.hpp"

namespace chasm {

// ---------------------------------------------------------------------------
// Kernel registry: every compiled (dtype, N, M, G).
#define CHASM_DECL(T, N, M, G, CL) extern template const KernelSet* kernel_set<T, N, M, G, CL, 0>();
CHASM_SHAPES(CHASM_DECL)
#undef CHASM_DECL
#define CHASM_DECL_TILES(T, N, M, G, CL)                                  \
    extern template const KernelSet* kernel_set<T, N, M, G, CL, 1>();      \
    extern template const KernelSet* kernel_set<T, N, M, G, CL, 2>();
CHASM_TILED_SHAPES(CHASM_DECL_TILES)
#undef CHASM_DECL_TILES

static const std::vector<const KernelSet*>& registry()
{
    static const std::vector<const KernelSet*> all = [] {
        std::vector<const KernelSet*> v;
#define CHASM_REG(T, N, M, G, CL) v.push_back(kernel_set<T, N, M, G, CL, 0>());
        CHASM_SHAPES(CHASM_REG)
#undef CHASM_REG
#define CHASM_REG_TILES(T, N, M, G, CL)                \
    v.push_back(kernel_set<T, N, M, G, CL, 1>());      \
    v.push_back(kernel_set<T, N, M, G, CL, 2>());
        CHASM_TILED_SHAPES(CHASM_REG_TILES)
#undef CHASM_REG_TILES
        return v;
    }();
    return all;
}

// The compiled kernels of (dtype, N, M, g, closure), or nullptr.
static const KernelSet* find_kernels(int dtype, int N, int M, int g, int closure, int tile)
{
    for (const KernelSet* k : registry())
        if (k->dtype == dtype && k->N == N && k->M == M && k->G == g && k->CL == closure && k->tile == tile)
            return k;
    return nullptr;
}

static int desc_tile(const chasm_advect_desc* d)
{
    return (int)((d->flags & CHASM_FLAG_TILE_MASK) >> CHASM_FLAG_TILE_SHIFT);
}

// Marker of the runtime-shape kernels (chasm_rt.hpp): descriptors without compiled
// kernels, the Hermite closure, or CHASM_FLAG_RUNTIME_SHAPE.
static const KernelSet kRuntimeKernels = {};
static bool is_rt(const KernelSet* ks) { return ks == &kRuntimeKernels; }

// Geometry of the runtime-shape kernels for a descriptor (no tables).
static RtJob rt_geometry(const chasm_advect_desc* d)
{
    RtJob j{};
    j.nitems = (long long)d->nbatch * d->nk[0] * d->nk[1] * d->nk[2];
    for (int a = 0; a < 3; ++a) {
        j.nx[a] = d->nx[a];
        j.nk[a] = d->nk[a];
        RtAxis& A = j.ax[a];
        A.N = d->nx[a];
        A.M = d->patch[a] < d->nx[a] - 1 ? d->patch[a] : (d->nx[a] - 1 > 0 ? d->nx[a] - 1 : 1);
        A.P = (A.N - 1 + A.M - 1) / A.M;
        A.MLAST = A.N - 1 - (A.P - 1) * A.M;
        A.G = d->ghost;
        A.poly3 = d->closure == CHASM_CLOSURE_POLY3;
    }
    return j;
}

// ---------------------------------------------------------------------------
// First stage of a long partial-row reduction: block (c, b) sums its fixed chunk of
// the rows of batch member b (strided over the threads, then a tree), so the result
// does not depend on timing.  The finalize kernel then reduces FOLD_CHUNKS rows.
constexpr int FOLD_CHUNKS = 256;
constexpr long long FOLD_MIN_ROWS = 4096;

__global__ __launch_bounds__(256) void k_fold(const double* __restrict__ in, long long rows, double* __restrict__ out)
{
    __shared__ double red[256][NRED];
    const long long per = (rows + gridDim.x - 1) / gridDim.x;
    const long long r0 = (long long)blockIdx.x * per;
    const long long r1 = r0 + per < rows ? r0 + per : rows;
    const double* p = in + (long long)blockIdx.y * rows * NRED;
    double acc[NRED];
    for (int v = 0; v < NRED; ++v) acc[v] = 0.0;
    for (long long r = r0 + threadIdx.x; r < r1; r += 256)
        for (int v = 0; v < NRED; ++v) acc[v] += p[r * NRED + v];
    for (int v = 0; v < NRED; ++v) red[threadIdx.x][v] = acc[v];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int v = 0; v < NRED; ++v) red[threadIdx.x][v] += red[threadIdx.x + w][v];
        __syncthreads();
    }
    if (threadIdx.x < NRED) out[((long long)blockIdx.y * gridDim.x + blockIdx.x) * NRED + threadIdx.x] = red[0][threadIdx.x];
}

__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, long long rows_per_batch,
                                                  FinalizeArgs a, double* __restrict__ out,
                                                  double* __restrict__ hist, int* __restrict__ counter,
                                                  int hist_cap, int nbatch)
{
    __shared__ double red[256][NRED];
    __shared__ int slot;
    if (threadIdx.x == 0) slot = hist ? (*counter % hist_cap) : 0;
    __syncthreads();
    for (int b = 0; b < nbatch; ++b) {
        double acc[NRED];
        for (int v = 0; v < NRED; ++v) acc[v] = 0.0;
        const double* p = partials + (long long)b * rows_per_batch * NRED;
        for (long long r = threadIdx.x; r < rows_per_batch; r += 256)
            for (int v = 0; v < NRED; ++v) acc[v] += p[r * NRED + v];
        for (int v = 0; v < NRED; ++v) red[threadIdx.x][v] = acc[v];
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if ((int)threadIdx.x < w)
                for (int v = 0; v < NRED; ++v) red[threadIdx.x][v] += red[threadIdx.x + w][v];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double* S = red[0];
            double r[NRED];
            r[0] = a.vol * S[0];
            r[1] = a.vol * S[1];
            for (int d = 0; d < 3; ++d) {
                r[2 + d] = a.vol * (a.xlo[d] * S[0] + a.hx[d] * S[2 + d]);
                r[5 + d] = a.vol * (a.klo[d] * S[0] + a.hk[d] * S[5 + d]);
            }
            for (int v = 0; v < NRED; ++v) out[b * NRED + v] = r[v];
            if (hist)
                for (int v = 0; v < NRED; ++v) hist[((long long)slot * nbatch + b) * NRED + v] = r[v];
        }
        __syncthreads();
    }
    if (hist && threadIdx.x == 0) *counter = *counter + 1;
}

// ---------------------------------------------------------------------------
// Fixed device workspace of chasm_advect_diagnostics_noalloc: per-item partial rows,
// fold rows and the finalized results of one call.  Each device holds its own copy
// for the life of the process.  Host code never passes `scratch` itself to a kernel
// (in host code the name is only a stand-in for the device array): it takes the
// array's device address, per device, from hipGetSymbolAddress and uses that.
constexpr size_t kNoAllocBytes = 16u << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up once per device).
static hipError_t noalloc_scratch(void** ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = p;
    }
    *ptr = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace chasm

using namespace chasm;

// ---------------------------------------------------------------------------
// Handle.
struct chasm_advect_s {
    chasm_advect_desc desc;
    void* f = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    const KernelSet* ks = nullptr;
    int schedule = CHASM_SCHED_AUTO;
    Work work{};                     // one-job work list of this handle, in place (f -> f)
    void* stage = nullptr;           // second field (CHASM_FLAG_OUT_OF_PLACE)
    Work w_fs{}, w_sf{}, w_ss{};     // f -> stage, stage -> f, stage -> stage
    FinalizeArgs fin{};
    void* tables = nullptr;          // device block: FP64 tables then FP32 mirror, int shifts
    double* partials = nullptr;      // [rows][NRED]
    double* fold = nullptr;          // [nbatch][FOLD_CHUNKS][NRED]
    double* marg_part = nullptr;     // item rows of the marginals (allocated on first use, or at
    double* marg_out = nullptr;      //   create with CHASM_FLAG_OBSERVE)
    bool observed = false;           // marg_out holds the observables of the last step call
    long long partial_rows = 0;      // rows per batch member when reducing each step
    double* last = nullptr;          // [nbatch][NRED]
    double* hist = nullptr;          // [cap][nbatch][NRED]
    int* counter = nullptr;
    int hist_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph2 = nullptr;     // two cube steps f -> stage -> f (CHASM_FLAG_OUT_OF_PLACE)
    hipGraphExec_t gexec2 = nullptr;
    hipGraph_t graphk = nullptr;     // kGraphSteps steps in one graph
    hipGraphExec_t gexeck = nullptr;
    hipGraph_t graph_r = nullptr;    // one CUBE step visiting the items last to first
    hipGraphExec_t gexec_r = nullptr;
    // SLAB pass sequences (see SlabSeq): one step, head, one and four middle units,
    // the two tails
    hipGraph_t sgraph[6] = {};
    hipGraphExec_t sgexec[6] = {};
    bool rev_next = false;           // the next CUBE step of chasm_advect_step visits in reverse
    hipStream_t cap_stream = nullptr;
    bool poisoned = false;
    // runtime-shape kernels: the job of each launch of a step (in place: all f -> f;
    // out of place: f -> stage, stage -> stage, stage -> f)
    bool rt = false;
    RtJob rtj[3] = {};
};

static thread_local std::string g_err;

namespace chasm {
long long marginal_row(const int nx[3]);
hipError_t launch_marginals(int dtype, const int nx[3], const int nk[3], int nbatch, const double hx[3],
                            const double hk[3], const void* f, double* part, double* out, hipStream_t st);

// The other C entry points of the library (chasm_theta.h) report through the same
// thread-local message.
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace chasm

static chasm_status fail(chasm_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

static chasm_status hip_fail(chasm_advect_t h, hipError_t e, const char* what)
{
    if (h) h->poisoned = true;
    return fail(CHASM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static chasm_status validate(const chasm_advect_desc* d, const KernelSet** ks_out)
{
    if (!d) return fail(CHASM_EINVAL, "desc is NULL");
    for (int i = 0; i < 3; ++i) {
        if (d->nx[i] < 2) return fail(CHASM_EINVAL, "nx must be >= 2 on every axis");
        if (d->nk[i] < 1) return fail(CHASM_EINVAL, "nk must be >= 1 on every axis");
        if (!(d->x_hi[i] > d->x_lo[i]) || !std::isfinite(d->x_lo[i]) || !std::isfinite(d->x_hi[i]))
            return fail(CHASM_EINVAL, "x extents must be finite with x_hi > x_lo");
        if (!(d->k_hi[i] > d->k_lo[i]) || !std::isfinite(d->k_lo[i]) || !std::isfinite(d->k_hi[i]))
            return fail(CHASM_EINVAL, "k extents must be finite with k_hi > k_lo");
        if (d->patch[i] < 1) return fail(CHASM_EINVAL, "patch must be >= 1");
    }
    if (d->ghost < 1) return fail(CHASM_EINVAL, "ghost must be >= 1");
    if (!std::isfinite(d->dt)) return fail(CHASM_EINVAL, "dt must be finite");
    if (d->dtype != CHASM_F32 && d->dtype != CHASM_F64) return fail(CHASM_EINVAL, "unknown dtype");
    if (d->closure < CHASM_CLOSURE_PMBC || d->closure > CHASM_CLOSURE_HERMITE) return fail(CHASM_EINVAL, "unknown closure");
    if (d->closure == CHASM_CLOSURE_POLY3 && d->ghost < 3) return fail(CHASM_EINVAL, "POLY3 closure needs ghost >= 3");
    if (d->closure == CHASM_CLOSURE_HERMITE)
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(d->slope_lo[i]) || !std::isfinite(d->slope_hi[i]))
                return fail(CHASM_EINVAL, "HERMITE closure needs finite end slopes");
    if (d->nbatch < 1) return fail(CHASM_EINVAL, "nbatch must be >= 1");
    if (d->schedule < CHASM_SCHED_AUTO || d->schedule > CHASM_SCHED_PLAIN) return fail(CHASM_EINVAL, "unknown schedule");
    if (d->history_cap < 0) return fail(CHASM_EINVAL, "history_cap must be >= 0");
    if (d->flags & ~(uint32_t)(CHASM_FLAG_REDUCE_EACH_STEP | CHASM_FLAG_GRAPH | CHASM_FLAG_OUT_OF_PLACE |
                               CHASM_FLAG_RUNTIME_SHAPE | CHASM_FLAG_TILE_MASK | CHASM_FLAG_OBSERVE))
        return fail(CHASM_EINVAL, "unknown flags");
    const int tile = desc_tile(d);
    if (tile >= kTiles) return fail(CHASM_EINVAL, "unknown tile variant");
    const double items = (double)d->nbatch * d->nk[0] * d->nk[1] * d->nk[2];
    const bool cubic = d->nx[0] == d->nx[1] && d->nx[0] == d->nx[2] && d->patch[0] == d->patch[1] &&
                       d->patch[0] == d->patch[2];
    const bool want_rt = (d->flags & CHASM_FLAG_RUNTIME_SHAPE) || d->closure == CHASM_CLOSURE_HERMITE;
    const KernelSet* ks = (cubic && !want_rt)
                              ? find_kernels(d->dtype, d->nx[0], d->patch[0], d->ghost, d->closure, tile)
                              : nullptr;
    if (tile > 0) {
        if (!ks)
            return fail(CHASM_EUNSUPPORTED, "tile variants exist only for compiled FP32 48^3 and 64^3 shapes");
        if (d->schedule == CHASM_SCHED_CUBE || d->schedule == CHASM_SCHED_AUTO)
            return fail(CHASM_EUNSUPPORTED, "a tile variant needs the SLAB or PLAIN schedule named");
    }
    if (ks) {
        if (d->schedule == CHASM_SCHED_CUBE && !ks->cube)
            return fail(CHASM_EUNSUPPORTED, "the x-cube does not fit in LDS for this nx and dtype");
        if (items * d->nx[0] > 2.0e9) return fail(CHASM_EUNSUPPORTED, "too many items for one launch grid");
    } else {
        // the runtime-shape kernels: resource limits only
        if (d->schedule == CHASM_SCHED_CUBE || d->schedule == CHASM_SCHED_SLAB)
            return fail(CHASM_EUNSUPPORTED, "no compiled kernels for this shape: the runtime-shape kernels run the "
                                            "PLAIN schedule (AUTO or PLAIN)");
        const RtJob g = rt_geometry(d);
        const int eb = d->dtype == CHASM_F64 ? 8 : 4;
        for (int a = 0; a < 3; ++a) {
            const int L = rt_lines_per_block(g, a, eb);
            if (L == 0) {
                char buf[200];
                std::snprintf(buf, sizeof buf, "axis %d: a line of %d nodes with patches of %d cells exceeds the LDS "
                              "tiles of the runtime-shape kernels", a + 1, d->nx[a], d->patch[a]);
                return fail(CHASM_EUNSUPPORTED, buf);
            }
            const double lines = (double)d->nx[0] * d->nx[1] * d->nx[2] / d->nx[a];
            if (items * std::ceil(lines / L) > 2.0e9) return fail(CHASM_EUNSUPPORTED, "too many blocks for one launch grid");
        }
        ks = &kRuntimeKernels;
    }
    if (ks_out) *ks_out = ks;
    return CHASM_OK;
}

static int resolve_schedule(const chasm_advect_desc* d, const KernelSet* ks)
{
    if (is_rt(ks)) return CHASM_SCHED_PLAIN;
    if (d->schedule != CHASM_SCHED_AUTO) return d->schedule;
    return ks->cube ? CHASM_SCHED_CUBE : CHASM_SCHED_SLAB;
}

// Rows of FP64 partials per batch member that a fused reduction of schedule sched can
// write (the largest over the passes that end a step).
static long long step_partial_rows(const chasm_advect_desc* d, const KernelSet* ks, int sched)
{
    const long long nkp = (long long)d->nk[0] * d->nk[1] * d->nk[2];
    if (is_rt(ks)) return nkp * rt_rows_per_item(rt_geometry(d), d->dtype);
    if (sched == CHASM_SCHED_CUBE) return nkp * ks->cube_rows;
    if (sched == CHASM_SCHED_SLAB) return nkp * std::max(ks->pencil_rows, ks->slab_rows);
    return nkp * ks->pencil_rows;
}

// Device table block: per axis the FP64 shift weights, their FP32 mirror and the
// integer shift classes.  (Stencil rows and patch factors are compile-time constants
// of the kernels; the host builds the stencil rows too, for the record and the tests.)
struct TableBlock {
    std::vector<char> bytes;
    size_t off_w64[3], off_w32[3], off_shift[3];
    // runtime-shape kernels: interface rows times h, end-slope bias times h, patch factors
    size_t off_st64[3], off_st32[3], off_bi64[3], off_bi32[3], off_lu64[3], off_lu32[3];
};

template <typename V>
static size_t push(std::vector<char>& b, const V* p, size_t n)
{
    size_t off = (b.size() + 255) & ~(size_t)255;
    b.resize(off + n * sizeof(V));
    std::memcpy(b.data() + off, p, n * sizeof(V));
    return off;
}

// FP64 vector and its FP32 mirror into the block.
static void push_both(std::vector<char>& b, const std::vector<double>& v, size_t& off64, size_t& off32)
{
    off64 = push(b, v.data(), v.size());
    const std::vector<float> f(v.begin(), v.end());
    off32 = push(b, f.data(), f.size());
}

static bool build_tables(const chasm_advect_desc* d, const KernelSet* ks, TableBlock& tb, std::string& err)
{
    const bool rt = is_rt(ks);
    const RtJob geo = rt_geometry(d);
    AxisTables at[3];
    for (int a = 0; a < 3; ++a) {
        const double h = (d->x_hi[a] - d->x_lo[a]) / d->nx[a];
        const double hk = (d->k_hi[a] - d->k_lo[a]) / d->nk[a];
        const int M = rt ? geo.ax[a].M : d->patch[a];
        if (!build_axis_tables(d->nx[a], M, d->ghost, rt ? d->ghost : ks->G, h, d->closure, d->nk[a], d->k_lo[a], hk,
                               d->dt, at[a], err, d->slope_lo[a], d->slope_hi[a]))
            return false;
    }
    for (int a = 0; a < 3; ++a) {
        tb.off_w64[a] = push(tb.bytes, at[a].w.data(), at[a].w.size());
        std::vector<float> w32(at[a].w.begin(), at[a].w.end());
        tb.off_w32[a] = push(tb.bytes, w32.data(), w32.size());
        tb.off_shift[a] = push(tb.bytes, at[a].shift.data(), at[a].shift.size());
        if (!rt) continue;
        const AxisTables& t = at[a];
        std::vector<double> st(t.stencil), bi(t.bias), lu((size_t)6 * (t.M + 1), 0.0);
        for (double& x : st) x *= t.h;
        for (double& x : bi) x *= t.h;
        const int ms[2] = {t.M, t.MLAST};
        for (int v = 0; v < 2; ++v) {
            double* base = lu.data() + (size_t)v * 3 * (t.M + 1);
            patch_factors(ms[v], base, base + (t.M + 1), base + 2 * (t.M + 1));
        }
        push_both(tb.bytes, st, tb.off_st64[a], tb.off_st32[a]);
        push_both(tb.bytes, bi, tb.off_bi64[a], tb.off_bi32[a]);
        push_both(tb.bytes, lu, tb.off_lu64[a], tb.off_lu32[a]);
    }
    return true;
}

static size_t field_bytes(const chasm_advect_desc* d)
{
    const size_t pts = (size_t)d->nbatch * d->nk[0] * d->nk[1] * d->nk[2] * d->nx[0] * d->nx[1] * d->nx[2];
    return pts * (d->dtype == CHASM_F64 ? sizeof(double) : sizeof(float));
}

// Bytes of the observables' item rows and of their sums (marginals and
// CHASM_FLAG_OBSERVE).
static std::pair<size_t, size_t> observe_bytes(const chasm_advect_desc* d)
{
    const long long nitems = (long long)d->nk[0] * d->nk[1] * d->nk[2] * d->nbatch;
    const long long per_b = (long long)d->nx[0] * d->nk[0] + (long long)d->nx[1] * d->nk[1] +
                            (long long)d->nx[2] * d->nk[2] + (long long)d->nx[0] * d->nx[1];
    return {(size_t)nitems * marginal_row(d->nx) * sizeof(double), (size_t)per_b * d->nbatch * sizeof(double)};
}

static size_t workspace_bytes(const chasm_advect_desc* d, const KernelSet* ks, int sched, size_t table_bytes)
{
    const long long nkp = (long long)d->nk[0] * d->nk[1] * d->nk[2];
    const bool red = (d->flags & CHASM_FLAG_REDUCE_EACH_STEP) != 0;
    const long long rows = (red ? std::max(step_partial_rows(d, ks, sched), nkp) : nkp) * d->nbatch;
    const int cap = d->history_cap > 0 ? d->history_cap : 1024;
    size_t b = table_bytes + 256;
    b += (size_t)rows * NRED * sizeof(double) + 256;
    b += (size_t)d->nbatch * FOLD_CHUNKS * NRED * sizeof(double) + 256;
    b += (size_t)d->nbatch * NRED * sizeof(double) + 256;
    if (d->flags & CHASM_FLAG_REDUCE_EACH_STEP) b += (size_t)cap * d->nbatch * NRED * sizeof(double) + 256 + 256;
    if (d->flags & CHASM_FLAG_OUT_OF_PLACE) b += field_bytes(d) + 256;
    if (d->flags & CHASM_FLAG_OBSERVE) b += observe_bytes(d).first + observe_bytes(d).second + 512;
    return b;
}

// Launch one step of schedule sched (CUBE or PLAIN) on stream s; pw[p] is the work
// list of the step's p-th launch (CUBE uses pw[0], PLAIN pw[0..2]).
static hipError_t launch_step(const KernelSet* ks, int sched, const Work* const pw[3], double* part, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (sched == CHASM_SCHED_CUBE) {
        e = ks->cube(*pw[0], part, s);
    } else {
        e = ks->slab[SLAB_X1](*pw[0], nullptr, s);
        if (e == hipSuccess) e = ks->pencil_x2(*pw[1], nullptr, s);
        if (e == hipSuccess) e = ks->pencil_x3(*pw[2], part, s);
    }
    return e;
}

// ---------------------------------------------------------------------------
// SLAB schedule.  A call of K steps alternates the sweep order between steps (x1 x2 x3,
// then x3 x2 x1, ...; the axis operators commute, see SlabMode), so it runs K + 1
// passes: pass r is
//   r = 0                      slab  x1 x2
//   r odd,  r < K              pencil x3 x3   (ends step r)
//   r even, 0 < r < K          slab  x2 x1 | x1 x2   (ends step r)
//   r = K odd                  pencil x3      (ends step K)
//   r = K even                 slab  x2 x1    (ends step K)
// Every pass but the first ends exactly one step, and a call always ends with the
// field after its last step.
enum PassKind { PASS_SLAB_A = 0, PASS_SLAB_B, PASS_SLAB_C, PASS_PENCIL_1, PASS_PENCIL_2 };

static int slab_pass_kind(int r, int K)
{
    if (r == 0) return PASS_SLAB_A;
    if (r % 2) return r == K ? PASS_PENCIL_1 : PASS_PENCIL_2;
    return r == K ? PASS_SLAB_C : PASS_SLAB_B;
}

static bool pass_is_slab(int kind) { return kind <= PASS_SLAB_C; }

static hipError_t launch_pass(const KernelSet* ks, int kind, const Work& w, double* part, hipStream_t s)
{
    switch (kind) {
    case PASS_SLAB_A: return ks->slab[SLAB_X1X2](w, nullptr, s);
    case PASS_SLAB_B: return ks->slab[SLAB_X2X1X1X2](w, part, s);
    case PASS_SLAB_C: return ks->slab[SLAB_X2X1](w, part, s);
    case PASS_PENCIL_1: return ks->pencil_x3(w, part, s);
    default: return ks->pencil_x3x3(w, part, s);
    }
}

// The work lists of one step of a handle.  In place, every launch reads and writes f.
// Out of place, the first launch reads f and writes the stage field and the last one
// reads the stage field and writes f (a middle PLAIN launch works on the stage field in
// place), so a step still ends in f.  CUBE has a single launch per step: its
// out-of-place form is the two-step pair of issue_cube_pair.
static void step_passes(const chasm_advect_s* h, const Work* pw[3])
{
    if (!h->stage || h->schedule == CHASM_SCHED_CUBE) {
        pw[0] = pw[1] = pw[2] = &h->work;
    } else {
        pw[0] = &h->w_fs;
        pw[1] = &h->w_ss;
        pw[2] = &h->w_sf;
    }
}

// Work list of a SLAB pass.  Out of place, slab passes that continue into a pencil read
// f and write the stage field and pencils read the stage field and write f; the closing
// x2 x1 slab runs in place on f.
static const Work* slab_pass_work(const chasm_advect_s* h, int kind)
{
    if (!h->stage || kind == PASS_SLAB_C) return &h->work;
    return pass_is_slab(kind) ? &h->w_fs : &h->w_sf;
}

// Issue one step's kernels of one handle on stream s.
// Reduce `rows` partial rows per batch member into the diagnostics (and, when
// `record`, the next history slot): one block directly, or a fold stage first.
static hipError_t launch_finalize(chasm_advect_s* h, long long rows, bool record, hipStream_t s)
{
    const double* src = h->partials;
    const int nb = h->desc.nbatch;
    if (rows > FOLD_MIN_ROWS) {
        hipLaunchKernelGGL(k_fold, dim3(FOLD_CHUNKS, nb), dim3(256), 0, s, h->partials, rows, h->fold);
        src = h->fold;
        rows = FOLD_CHUNKS;
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, src, rows, h->fin, h->last, record ? h->hist : nullptr,
                       record ? h->counter : nullptr, record ? h->hist_cap : 1, nb);
    return hipGetLastError();
}

// rev: a CUBE step visits the items last to first.  chasm_advect_step alternates the
// order from step to step, so the items a step stores last are the first ones the next
// step loads, while they may still sit in the memory-side cache.
static hipError_t issue_passes(chasm_advect_t h, hipStream_t s, const int* kinds, int n);

static hipError_t issue_step(chasm_advect_t h, hipStream_t s, bool rev = false)
{
    if (h->rt) {
        const bool red = (h->desc.flags & CHASM_FLAG_REDUCE_EACH_STEP) != 0;
        hipError_t e = hipSuccess;
        for (int a = 0; a < 3 && e == hipSuccess; ++a)
            e = rt_sweep(h->rtj[a], a, h->desc.dtype, (red && a == 2) ? h->partials : nullptr, s);
        if (e == hipSuccess && red) e = launch_finalize(h, h->partial_rows, true, s);
        return e;
    }
    if (h->schedule == CHASM_SCHED_SLAB) {
        const int one[2] = {PASS_SLAB_A, PASS_PENCIL_1};
        return issue_passes(h, s, one, 2);
    }
    const bool red = (h->desc.flags & CHASM_FLAG_REDUCE_EACH_STEP) != 0;
    double* part = red ? h->partials : nullptr;
    const Work* pw[3];
    step_passes(h, pw);
    Work wr;
    if (rev && h->schedule == CHASM_SCHED_CUBE) {
        wr = *pw[0];
        for (int j = 0; j < wr.njobs; ++j) wr.jobs[j].reverse = 1;
        pw[0] = pw[1] = pw[2] = &wr;
    }
    hipError_t e = launch_step(h->ks, h->schedule, pw, part, s);
    if (e == hipSuccess && red) e = launch_finalize(h, h->partial_rows, true, s);
    return e;
}

// Issue SLAB passes of the given kinds on stream s, each pass that ends a step followed
// by its reduction when the handle records per-step diagnostics.
static hipError_t issue_passes(chasm_advect_t h, hipStream_t s, const int* kinds, int n)
{
    const bool red = (h->desc.flags & CHASM_FLAG_REDUCE_EACH_STEP) != 0;
    const long long nkp = (long long)h->desc.nk[0] * h->desc.nk[1] * h->desc.nk[2];
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const int kind = kinds[i];
        const bool ends = red && kind != PASS_SLAB_A;
        e = launch_pass(h->ks, kind, *slab_pass_work(h, kind), ends ? h->partials : nullptr, s);
        if (e == hipSuccess && ends)
            e = launch_finalize(h, nkp * (pass_is_slab(kind) ? h->ks->slab_rows : h->ks->pencil_rows), true, s);
    }
    return e;
}

// SLAB graph slots and their pass lists.
enum { SG_ONE = 0, SG_HEAD, SG_MID1, SG_MID4, SG_TAIL_EVEN, SG_TAIL_ODD, SG_COUNT };
static int slab_graph_passes(int g, int* kinds)
{
    switch (g) {
    case SG_ONE: kinds[0] = PASS_SLAB_A; kinds[1] = PASS_PENCIL_1; return 2;
    case SG_HEAD: kinds[0] = PASS_SLAB_A; kinds[1] = PASS_PENCIL_2; return 2;
    case SG_MID1: kinds[0] = PASS_SLAB_B; kinds[1] = PASS_PENCIL_2; return 2;
    case SG_MID4:
        for (int i = 0; i < 4; ++i) {
            kinds[2 * i] = PASS_SLAB_B;
            kinds[2 * i + 1] = PASS_PENCIL_2;
        }
        return 8;
    case SG_TAIL_EVEN: kinds[0] = PASS_SLAB_C; return 1;
    default: kinds[0] = PASS_SLAB_B; kinds[1] = PASS_PENCIL_1; return 2;
    }
}

// K steps of a SLAB handle: K + 1 passes (slab_pass_kind), as graph replays when the
// handle has them.
static hipError_t slab_steps(chasm_advect_t h, hipStream_t s, int K)
{
    if (K <= 0) return hipSuccess;
    auto run = [&](int g) {
        if (h->sgexec[g]) return hipGraphLaunch(h->sgexec[g], s);
        int kinds[8];
        const int n = slab_graph_passes(g, kinds);
        return issue_passes(h, s, kinds, n);
    };
    if (K == 1) return run(SG_ONE);
    hipError_t e = run(SG_HEAD);
    const int mid = (K % 2 == 0) ? (K - 2) / 2 : (K - 3) / 2;
    for (int i = 0; i < mid / 4 && e == hipSuccess; ++i) e = run(SG_MID4);
    for (int i = 0; i < mid % 4 && e == hipSuccess; ++i) e = run(SG_MID1);
    if (e == hipSuccess) e = run(K % 2 == 0 ? SG_TAIL_EVEN : SG_TAIL_ODD);
    return e;
}

// Two CUBE steps out of place: f -> stage (first item first), then stage -> f (last
// item first).
static hipError_t issue_cube_pair(chasm_advect_t h, hipStream_t s)
{
    const bool red = (h->desc.flags & CHASM_FLAG_REDUCE_EACH_STEP) != 0;
    double* part = red ? h->partials : nullptr;
    Work back = h->w_sf;
    back.jobs[0].reverse = 1;
    const Work* first[3] = {&h->w_fs, &h->w_fs, &h->w_fs};
    const Work* second[3] = {&back, &back, &back};
    hipError_t e = launch_step(h->ks, CHASM_SCHED_CUBE, first, part, s);
    if (e == hipSuccess && red) e = launch_finalize(h, h->partial_rows, true, s);
    if (e == hipSuccess) e = launch_step(h->ks, CHASM_SCHED_CUBE, second, part, s);
    if (e == hipSuccess && red) e = launch_finalize(h, h->partial_rows, true, s);
    return e;
}

static bool cube_pairs(const chasm_advect_s* h) { return h->stage && h->schedule == CHASM_SCHED_CUBE; }

// The sums of the observables from the item rows in marg_part; with f given, the
// separate pass forms the rows from that field first.
static hipError_t launch_observables(chasm_advect_s* h, const void* f, hipStream_t s)
{
    const chasm_advect_desc& d = h->desc;
    double hx[3], hk[3];
    for (int a = 0; a < 3; ++a) {
        hx[a] = (d.x_hi[a] - d.x_lo[a]) / d.nx[a];
        hk[a] = (d.k_hi[a] - d.k_lo[a]) / d.nk[a];
    }
    return launch_marginals(d.dtype, d.nx, d.nk, d.nbatch, hx, hk, f, h->marg_part, h->marg_out, s);
}

// The last step of an observed call (CHASM_FLAG_OBSERVE): x1, x2, x3 as three launches
// (the PLAIN form of every schedule's kernels), the x3 launch writing the observables'
// item rows in its epilogue, then their sums.  Runtime-shape lines the fast kernel form
// does not serve take the separate row pass instead.  With per-step diagnostics, the
// step's row comes from a reduction of the stored field.
static hipError_t issue_observed_step(chasm_advect_t h, hipStream_t s)
{
    const bool red = (h->desc.flags & CHASM_FLAG_REDUCE_EACH_STEP) != 0;
    const int dt = h->desc.dtype;
    hipError_t e = hipSuccess;
    bool fused = true;
    if (h->rt) {
        for (int a = 0; a < 2 && e == hipSuccess; ++a) e = rt_sweep(h->rtj[a], a, dt, nullptr, s);
        fused = rt_can_observe(h->rtj[2], dt);
        if (e == hipSuccess)
            e = fused ? rt_sweep_obs(h->rtj[2], dt, h->marg_part, s) : rt_sweep(h->rtj[2], 2, dt, nullptr, s);
        if (e == hipSuccess && red) e = rt_reduce(h->rtj[0], dt, h->partials, s);
    } else {
        const Work* pw[3];
        step_passes(h, pw);
        e = h->ks->slab[SLAB_X1](*pw[0], nullptr, s);
        if (e == hipSuccess) e = h->ks->pencil_x2(*pw[1], nullptr, s);
        if (e == hipSuccess) e = h->ks->pencil_x3_obs(*pw[2], h->marg_part, s);
        if (e == hipSuccess && red) e = h->ks->reduce(h->work, h->partials, s);
    }
    if (e == hipSuccess && red)
        e = launch_finalize(h, (long long)h->desc.nk[0] * h->desc.nk[1] * h->desc.nk[2], true, s);
    if (e == hipSuccess) e = launch_observables(h, fused ? nullptr : h->f, s);
    return e;
}

// Steps per graph launch for long step counts (CHASM_FLAG_GRAPH): one launch per step
// leaves a few microseconds between consecutive graphs; within a graph the kernels
// follow each other directly.
constexpr int kGraphSteps = 8;

extern "C" {

const char* chasm_advect_last_error(void) { return g_err.c_str(); }

const char* chasm_advect_version(void) { return "chasm-advect 0.1 (gfx950)"; }

chasm_status chasm_advect_workspace_bytes(const chasm_advect_desc* desc, size_t* bytes)
{
    const KernelSet* ks = nullptr;
    chasm_status st = validate(desc, &ks);
    if (st != CHASM_OK) return st;
    if (!bytes) return fail(CHASM_EINVAL, "bytes is NULL");
    TableBlock tb;
    std::string err;
    if (!build_tables(desc, ks, tb, err)) return fail(CHASM_EINVAL, err);
    *bytes = workspace_bytes(desc, ks, resolve_schedule(desc, ks), tb.bytes.size());
    return CHASM_OK;
}

chasm_status chasm_advect_create(const chasm_advect_desc* desc, void* f_dev, void* hip_stream, chasm_advect_t* out)
{
    if (!out) return fail(CHASM_EINVAL, "out is NULL");
    *out = nullptr;
    const KernelSet* ks = nullptr;
    chasm_status st = validate(desc, &ks);
    if (st != CHASM_OK) return st;
    if (!f_dev) return fail(CHASM_EINVAL, "f_dev is NULL");
    if (((uintptr_t)f_dev) % 16) return fail(CHASM_EINVAL, "f_dev must be 16-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, f_dev) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(CHASM_EINVAL, "f_dev is not a device pointer");
    }

    TableBlock tb;
    std::string err;
    if (!build_tables(desc, ks, tb, err)) return fail(CHASM_EINVAL, err);

    chasm_advect_s* h = new (std::nothrow) chasm_advect_s();
    if (!h) return fail(CHASM_ENOMEM, "host allocation failed");
    h->desc = *desc;
    h->f = f_dev;
    h->stream = (hipStream_t)hip_stream;
    h->ks = ks;
    h->schedule = resolve_schedule(desc, ks);
    hipGetDevice(&h->device);

    auto bail = [&](chasm_status s, const std::string& m) {
        chasm_advect_destroy(h);
        return fail(s, m);
    };
    hipError_t e = hipMalloc(&h->tables, tb.bytes.size());
    if (e != hipSuccess) return bail(CHASM_ENOMEM, "hipMalloc(tables) failed");
    e = hipMemcpyAsync(h->tables, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return bail(CHASM_EDEVICE, "table upload failed");

    const long long nkp = (long long)desc->nk[0] * desc->nk[1] * desc->nk[2];
    h->partial_rows = step_partial_rows(desc, ks, h->schedule);
    // partial rows: one per item for diagnostics of the current field, and per block of
    // the passes that end a step when those reduce
    const bool red = (desc->flags & CHASM_FLAG_REDUCE_EACH_STEP) != 0;
    const long long rows = (red ? std::max(h->partial_rows, nkp) : nkp) * desc->nbatch;
    if (hipMalloc((void**)&h->partials, (size_t)rows * NRED * sizeof(double)) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(partials) failed");
    if (hipMalloc((void**)&h->fold, (size_t)desc->nbatch * FOLD_CHUNKS * NRED * sizeof(double)) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(fold) failed");
    if (desc->flags & CHASM_FLAG_OBSERVE) {
        const auto ob = observe_bytes(desc);
        if (hipMalloc((void**)&h->marg_part, ob.first) != hipSuccess ||
            hipMalloc((void**)&h->marg_out, ob.second) != hipSuccess)
            return bail(CHASM_ENOMEM, "hipMalloc(observable rows) failed");
    }
    if (hipMalloc((void**)&h->last, (size_t)desc->nbatch * NRED * sizeof(double)) != hipSuccess)
        return bail(CHASM_ENOMEM, "hipMalloc(diagnostics) failed");
    if (desc->flags & CHASM_FLAG_REDUCE_EACH_STEP) {
        h->hist_cap = desc->history_cap > 0 ? desc->history_cap : 1024;
        if (hipMalloc((void**)&h->hist, (size_t)h->hist_cap * desc->nbatch * NRED * sizeof(double)) != hipSuccess)
            return bail(CHASM_ENOMEM, "hipMalloc(history) failed");
        if (hipMalloc((void**)&h->counter, sizeof(int)) != hipSuccess)
            return bail(CHASM_ENOMEM, "hipMalloc(counter) failed");
        if (hipMemsetAsync(h->counter, 0, sizeof(int), h->stream) != hipSuccess)
            return bail(CHASM_EDEVICE, "counter reset failed");
    }

    const bool f64 = desc->dtype == CHASM_F64;
    char* tbase = static_cast<char*>(h->tables);
    JobDev& job = h->work.jobs[0];
    h->work.njobs = 1;
    h->work.first[0] = 0;
    h->work.first[1] = nkp * desc->nbatch;
    job.f = f_dev;
    job.out = f_dev;
    job.nitems = nkp * desc->nbatch;
    for (int a = 0; a < 3; ++a) {
        job.nk[a] = desc->nk[a];
        job.ax[a].w = tbase + (f64 ? tb.off_w64[a] : tb.off_w32[a]);
        job.ax[a].shift = reinterpret_cast<const int*>(tbase + tb.off_shift[a]);
        const double hx = (desc->x_hi[a] - desc->x_lo[a]) / desc->nx[a];
        h->fin.xlo[a] = desc->x_lo[a];
        h->fin.hx[a] = hx;
        h->fin.klo[a] = desc->k_lo[a];
        h->fin.hk[a] = (desc->k_hi[a] - desc->k_lo[a]) / desc->nk[a];
    }
    h->fin.vol = h->fin.hx[0] * h->fin.hx[1] * h->fin.hx[2] * h->fin.hk[0] * h->fin.hk[1] * h->fin.hk[2];

    if (desc->flags & CHASM_FLAG_OUT_OF_PLACE) {
        if (hipMalloc(&h->stage, field_bytes(desc)) != hipSuccess)
            return bail(CHASM_ENOMEM, "hipMalloc(stage field) failed");
        h->w_fs = h->w_sf = h->w_ss = h->work;
        h->w_fs.jobs[0].out = h->stage;
        h->w_sf.jobs[0].f = h->stage;
        h->w_ss.jobs[0].f = h->w_ss.jobs[0].out = h->stage;
    }
    if (is_rt(ks)) {
        h->rt = true;
        RtJob j = rt_geometry(desc);
        for (int a = 0; a < 3; ++a) {
            RtAxis& A = j.ax[a];
            A.stencil = tbase + (f64 ? tb.off_st64[a] : tb.off_st32[a]);
            A.bias = tbase + (f64 ? tb.off_bi64[a] : tb.off_bi32[a]);
            A.lu = tbase + (f64 ? tb.off_lu64[a] : tb.off_lu32[a]);
            A.shift = reinterpret_cast<const int*>(tbase + tb.off_shift[a]);
            A.w = tbase + (f64 ? tb.off_w64[a] : tb.off_w32[a]);
        }
        for (int p = 0; p < 3; ++p) {
            h->rtj[p] = j;
            h->rtj[p].f = f_dev;
            h->rtj[p].out = f_dev;
        }
        if (h->stage) {   // x1: f -> stage, x2: stage -> stage, x3: stage -> f
            h->rtj[0].out = h->stage;
            h->rtj[1].f = h->rtj[1].out = h->stage;
            h->rtj[2].f = h->stage;
        }
    }

    if (desc->flags & CHASM_FLAG_GRAPH) {
        if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return bail(CHASM_EDEVICE, "capture stream creation failed");
        // Capture `steps` steps (pairs when the CUBE steps run out of place) as one graph.
        auto capture = [&](int steps, hipGraph_t* g, hipGraphExec_t* x) {
            if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
            hipError_t ce = hipSuccess;
            for (int i = 0; i < steps && ce == hipSuccess;) {
                const bool pair = cube_pairs(h) && i + 1 < steps;
                ce = pair ? issue_cube_pair(h, h->cap_stream) : issue_step(h, h->cap_stream, (i % 2) == 1);
                i += pair ? 2 : 1;
            }
            const hipError_t ee = hipStreamEndCapture(h->cap_stream, g);
            return ce == hipSuccess && ee == hipSuccess && hipGraphInstantiate(x, *g, nullptr, nullptr, 0) == hipSuccess;
        };
        if (h->schedule == CHASM_SCHED_SLAB) {
            for (int g = 0; g < SG_COUNT; ++g) {
                int kinds[8];
                const int n = slab_graph_passes(g, kinds);
                if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return bail(CHASM_EDEVICE, "hipStreamBeginCapture failed");
                const hipError_t ce = issue_passes(h, h->cap_stream, kinds, n);
                const hipError_t ee = hipStreamEndCapture(h->cap_stream, &h->sgraph[g]);
                if (ce != hipSuccess || ee != hipSuccess ||
                    hipGraphInstantiate(&h->sgexec[g], h->sgraph[g], nullptr, nullptr, 0) != hipSuccess)
                    return bail(CHASM_EDEVICE, "pass-sequence capture failed");
            }
            *out = h;
            return CHASM_OK;
        }
        if (!capture(1, &h->graph, &h->gexec)) return bail(CHASM_EDEVICE, "step capture failed");
        if (h->schedule == CHASM_SCHED_CUBE) {   // the reversed single step
            if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return bail(CHASM_EDEVICE, "hipStreamBeginCapture failed");
            const hipError_t ce = issue_step(h, h->cap_stream, true);
            const hipError_t ee = hipStreamEndCapture(h->cap_stream, &h->graph_r);
            if (ce != hipSuccess || ee != hipSuccess ||
                hipGraphInstantiate(&h->gexec_r, h->graph_r, nullptr, nullptr, 0) != hipSuccess)
                return bail(CHASM_EDEVICE, "step capture failed");
        }
        if (cube_pairs(h) && !capture(2, &h->graph2, &h->gexec2)) return bail(CHASM_EDEVICE, "step-pair capture failed");
        if (!capture(kGraphSteps, &h->graphk, &h->gexeck)) return bail(CHASM_EDEVICE, "multi-step capture failed");
    }
    *out = h;
    return CHASM_OK;
}

static chasm_status steps_unobserved(chasm_advect_t h, int32_t nsteps);

chasm_status chasm_advect_step(chasm_advect_t h, int32_t nsteps)
{
    if (!h) return fail(CHASM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    if (nsteps < 0) return fail(CHASM_EINVAL, "nsteps must be >= 0");
    if (!(h->desc.flags & CHASM_FLAG_OBSERVE) || nsteps == 0) return steps_unobserved(h, nsteps);
    chasm_status st = steps_unobserved(h, nsteps - 1);
    if (st != CHASM_OK) return st;
    hipError_t e = issue_observed_step(h, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "observed step launch");
    h->observed = true;
    return CHASM_OK;
}

static chasm_status steps_unobserved(chasm_advect_t h, int32_t nsteps)
{
    if (h->schedule == CHASM_SCHED_SLAB) {
        hipError_t e = slab_steps(h, h->stream, nsteps);
        if (e != hipSuccess) return hip_fail(h, e, "step launch");
        return CHASM_OK;
    }
    const bool cube = h->schedule == CHASM_SCHED_CUBE;
    // One step in the current visiting order; the order alternates for CUBE.
    auto single = [&]() {
        const bool rev = cube && h->rev_next;
        hipError_t e = h->gexec ? hipGraphLaunch(rev ? h->gexec_r : h->gexec, h->stream) : issue_step(h, h->stream, rev);
        h->rev_next = cube && !h->rev_next;
        return e;
    };
    int32_t s = 0;
    if (h->rev_next && nsteps > 0) {   // realign: the multi-step graphs and pairs start forward
        hipError_t e = single();
        if (e != hipSuccess) return hip_fail(h, e, "step launch");
        s = 1;
    }
    // Even-length groups below keep the order's parity.
    if (h->gexeck)
        for (; s + kGraphSteps <= nsteps; s += kGraphSteps) {
            hipError_t e = hipGraphLaunch(h->gexeck, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "step launch");
        }
    if (cube_pairs(h))
        for (; s + 1 < nsteps; s += 2) {
            hipError_t e = h->gexec2 ? hipGraphLaunch(h->gexec2, h->stream) : issue_cube_pair(h, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "step launch");
        }
    for (; s < nsteps; ++s) {
        hipError_t e = single();
        if (e != hipSuccess) return hip_fail(h, e, "step launch");
    }
    return CHASM_OK;
}

chasm_status chasm_advect_step_many(const chasm_advect_t* hs, int32_t n, const int32_t* nsteps)
{
    if (n < 0 || (n > 0 && (!hs || !nsteps))) return fail(CHASM_EINVAL, "bad handle list");
    for (int32_t i = 0; i < n; ++i) {
        if (!hs[i]) return fail(CHASM_EINVAL, "NULL handle in list");
        if (hs[i]->poisoned) return fail(CHASM_ESTATE, "a handle in the list is poisoned");
        if (nsteps[i] < 0) return fail(CHASM_EINVAL, "nsteps must be >= 0");
        if (hs[i]->stream != hs[0]->stream) return fail(CHASM_EINVAL, "all handles must share one stream");
        for (int32_t j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return fail(CHASM_EINVAL, "a handle appears twice in the list");
    }
    hipStream_t s = n > 0 ? hs[0]->stream : nullptr;
    // Handles that record per-step diagnostics run their call on their own, exactly as
    // chasm_advect_step does.
    auto alone = [](chasm_advect_t h) {
        return (h->desc.flags & (CHASM_FLAG_REDUCE_EACH_STEP | CHASM_FLAG_OBSERVE)) || h->rt;
    };
    for (int32_t i = 0; i < n; ++i)
        if (alone(hs[i])) {
            const chasm_status st = chasm_advect_step(hs[i], nsteps[i]);
            if (st != CHASM_OK) return st;
        }
    // The others advance round by round: round r is step r of a CUBE or PLAIN handle and
    // pass r of a SLAB handle's K + 1 passes (slab_pass_kind), so every job progresses
    // together.  Handles with the same kernels, schedule and pass share one launch (work
    // lists of at most kMaxJobs jobs).
    constexpr int kStep = -1;
    auto kind_at = [&](int32_t i, int32_t r) -> int {   // what round r runs for handle i (-2: nothing)
        const int32_t K = nsteps[i];
        if (hs[i]->schedule == CHASM_SCHED_SLAB) return (K > 0 && r <= K) ? slab_pass_kind(r, K) : -2;
        return r < K ? kStep : -2;
    };
    int32_t rounds = 0;
    for (int32_t i = 0; i < n; ++i)
        if (!alone(hs[i]))
            rounds = std::max(rounds, hs[i]->schedule == CHASM_SCHED_SLAB && nsteps[i] > 0 ? nsteps[i] + 1 : nsteps[i]);
    std::vector<int32_t> live;
    std::vector<int> kinds;
    for (int32_t r = 0; r < rounds; ++r) {
        live.clear();
        kinds.clear();
        for (int32_t i = 0; i < n; ++i) {
            if (alone(hs[i])) continue;
            const int k = kind_at(i, r);
            if (k == -2) continue;
            live.push_back(i);
            kinds.push_back(k);
        }
        std::vector<bool> done(live.size(), false);
        for (size_t a = 0; a < live.size(); ++a) {
            if (done[a]) continue;
            chasm_advect_t h = hs[live[a]];
            const int kind = kinds[a];
            // One work list per launch; job j of list p is launch p of its handle's step
            // (in place, or through that handle's stage field).
            Work w[3] = {};
            for (size_t b = a; b < live.size() && w[0].njobs < kMaxJobs; ++b) {
                chasm_advect_t o = hs[live[b]];
                if (done[b] || o->ks != h->ks || o->schedule != h->schedule || kinds[b] != kind) continue;
                const long long items = o->work.jobs[0].nitems;
                if (w[0].first[w[0].njobs] + items > (1LL << 24)) break;   // keep launch grids small
                const Work* pw[3];
                if (kind == kStep) {
                    step_passes(o, pw);
                } else {
                    pw[0] = pw[1] = pw[2] = slab_pass_work(o, kind);
                }
                for (int p = 0; p < 3; ++p) {
                    w[p].jobs[w[p].njobs] = pw[p]->jobs[0];
                    w[p].first[w[p].njobs + 1] = w[p].first[w[p].njobs] + items;
                    ++w[p].njobs;
                }
                done[b] = true;
            }
            hipError_t e = hipSuccess;
            if (w[0].njobs == 0) {   // a single job larger than the per-launch bound
                if (kind == kStep) {
                    e = issue_step(h, s);
                } else {
                    e = launch_pass(h->ks, kind, *slab_pass_work(h, kind), nullptr, s);
                }
                done[a] = true;
            } else if (kind == kStep) {
                const Work* pw[3] = {&w[0], &w[1], &w[2]};
                e = launch_step(h->ks, h->schedule, pw, nullptr, s);
            } else {
                e = launch_pass(h->ks, kind, w[0], nullptr, s);
            }
            if (e != hipSuccess) return hip_fail(h, e, "batched step launch");
        }
    }
    return CHASM_OK;
}

chasm_status chasm_advect_diagnostics(chasm_advect_t h, double* out)
{
    if (!h || !out) return fail(CHASM_EINVAL, "NULL argument");
    if (h->poisoned) return fail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    hipError_t e = h->rt ? rt_reduce(h->rtj[0], h->desc.dtype, h->partials, h->stream)
                         : h->ks->reduce(h->work, h->partials, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "reduce launch");
    const long long nkp = (long long)h->desc.nk[0] * h->desc.nk[1] * h->desc.nk[2];
    e = launch_finalize(h, nkp, false, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "finalize launch");
    e = hipMemcpyAsync(out, h->last, (size_t)h->desc.nbatch * NRED * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "diagnostics copy");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    return CHASM_OK;
}

chasm_status chasm_advect_diagnostics_noalloc(const chasm_advect_desc* desc, const void* f_dev, void* hip_stream,
                                              double* out_dev)
{
    const KernelSet* ks = nullptr;
    chasm_status st = validate(desc, &ks);
    if (st != CHASM_OK) return st;
    if (!f_dev || !out_dev) return fail(CHASM_EINVAL, "f_dev and out_dev must be device pointers");
    if (((uintptr_t)f_dev) % 16) return fail(CHASM_EINVAL, "f_dev must be 16-byte aligned");
    const long long nkp = (long long)desc->nk[0] * desc->nk[1] * desc->nk[2];
    const long long items = nkp * desc->nbatch;
    // workspace: one FP64 partial row per item, the fold rows, the results
    const size_t part_b = ((size_t)items * NRED * sizeof(double) + 255) & ~(size_t)255;
    const size_t fold_b = ((size_t)desc->nbatch * FOLD_CHUNKS * NRED * sizeof(double) + 255) & ~(size_t)255;
    if (part_b + fold_b > kNoAllocBytes) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "%lld items need %zu bytes of partials, more than the %zu-byte no-allocation workspace",
                      items, part_b + fold_b, kNoAllocBytes);
        return fail(CHASM_EINVAL, buf);
    }
    void* ws = nullptr;
    hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess) return fail(CHASM_EDEVICE, std::string("workspace lookup: ") + hipGetErrorString(e));
    double* part = static_cast<double*>(ws);
    double* fold = reinterpret_cast<double*>(static_cast<char*>(ws) + part_b);
    hipStream_t s = (hipStream_t)hip_stream;

    Work w{};
    w.njobs = 1;
    w.first[0] = 0;
    w.first[1] = items;
    w.jobs[0].f = const_cast<void*>(f_dev);
    w.jobs[0].out = const_cast<void*>(f_dev);
    w.jobs[0].nitems = items;
    FinalizeArgs fin{};
    for (int a = 0; a < 3; ++a) {
        w.jobs[0].nk[a] = desc->nk[a];
        fin.xlo[a] = desc->x_lo[a];
        fin.hx[a] = (desc->x_hi[a] - desc->x_lo[a]) / desc->nx[a];
        fin.klo[a] = desc->k_lo[a];
        fin.hk[a] = (desc->k_hi[a] - desc->k_lo[a]) / desc->nk[a];
    }
    fin.vol = fin.hx[0] * fin.hx[1] * fin.hx[2] * fin.hk[0] * fin.hk[1] * fin.hk[2];
    // the same kernels and summation order as chasm_advect_diagnostics
    if (is_rt(ks)) {
        RtJob j = rt_geometry(desc);
        j.f = f_dev;
        e = rt_reduce(j, desc->dtype, part, s);
    } else {
        e = ks->reduce(w, part, s);
    }
    if (e != hipSuccess) return fail(CHASM_EDEVICE, std::string("reduce launch: ") + hipGetErrorString(e));
    const double* src = part;
    long long rows = nkp;
    if (rows > FOLD_MIN_ROWS) {
        hipLaunchKernelGGL(k_fold, dim3(FOLD_CHUNKS, desc->nbatch), dim3(256), 0, s, part, rows, fold);
        src = fold;
        rows = FOLD_CHUNKS;
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, src, rows, fin, out_dev, nullptr, nullptr, 1,
                       desc->nbatch);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(CHASM_EDEVICE, std::string("finalize launch: ") + hipGetErrorString(e));
    return CHASM_OK;
}

static chasm_status copy_observables(chasm_advect_t h, double* w1, double* w2, double* w3, double* p12);

chasm_status chasm_advect_marginals(chasm_advect_t h, double* w1, double* w2, double* w3, double* p12)
{
    if (!h) return fail(CHASM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    if (!h->marg_part) {
        const auto ob = observe_bytes(&h->desc);
        if (hipMalloc((void**)&h->marg_part, ob.first) != hipSuccess)
            return fail(CHASM_ENOMEM, "hipMalloc(marginal rows) failed");
        if (hipMalloc((void**)&h->marg_out, ob.second) != hipSuccess)
            return fail(CHASM_ENOMEM, "hipMalloc(marginals) failed");
    }
    hipError_t e = launch_observables(h, h->f, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "marginals launch");
    // the buffers now hold this field's marginals, not the last observed call's
    h->observed = false;
    return copy_observables(h, w1, w2, w3, p12);
}

chasm_status chasm_advect_observables(chasm_advect_t h, double* w1, double* w2, double* w3, double* p12)
{
    if (!h) return fail(CHASM_EINVAL, "handle is NULL");
    if (h->poisoned) return fail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    if (!(h->desc.flags & CHASM_FLAG_OBSERVE)) return fail(CHASM_EINVAL, "handle was created without CHASM_FLAG_OBSERVE");
    if (!h->observed) return fail(CHASM_EINVAL, "no observed step since create or the last marginals call");
    return copy_observables(h, w1, w2, w3, p12);
}

// Copy the sums in marg_out to the host arrays (stream-ordered, then synchronised).
static chasm_status copy_observables(chasm_advect_t h, double* w1, double* w2, double* w3, double* p12)
{
    const chasm_advect_desc& d = h->desc;
    const int N0 = d.nx[0], N1 = d.nx[1], N2 = d.nx[2];
    const long long per_b = (long long)N0 * d.nk[0] + (long long)N1 * d.nk[1] + (long long)N2 * d.nk[2] +
                            (long long)N0 * N1;
    hipError_t e;
    std::vector<double> all((size_t)per_b * d.nbatch);
    e = hipMemcpyAsync(all.data(), h->marg_out, all.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "marginals copy");
    const size_t n1 = (size_t)N0 * d.nk[0], n2 = (size_t)N1 * d.nk[1], n3 = (size_t)N2 * d.nk[2],
                 np = (size_t)N0 * N1;
    for (int b = 0; b < d.nbatch; ++b) {
        const double* src = all.data() + (size_t)b * per_b;
        if (w1) std::memcpy(w1 + b * n1, src, n1 * sizeof(double));
        if (w2) std::memcpy(w2 + b * n2, src + n1, n2 * sizeof(double));
        if (w3) std::memcpy(w3 + b * n3, src + n1 + n2, n3 * sizeof(double));
        if (p12) std::memcpy(p12 + b * np, src + n1 + n2 + n3, np * sizeof(double));
    }
    return CHASM_OK;
}

chasm_status chasm_advect_mass(chasm_advect_t h, double* mass, double* l2, double* moments6)
{
    if (!h || !mass) return fail(CHASM_EINVAL, "NULL argument");
    std::vector<double> all((size_t)h->desc.nbatch * NRED);
    chasm_status st = chasm_advect_diagnostics(h, all.data());
    if (st != CHASM_OK) return st;
    double s[NRED] = {0};
    for (int b = 0; b < h->desc.nbatch; ++b)
        for (int v = 0; v < NRED; ++v) s[v] += all[(size_t)b * NRED + v];
    *mass = s[0];
    if (l2) *l2 = s[1];
    if (moments6)
        for (int v = 0; v < 6; ++v) moments6[v] = s[2 + v];
    return CHASM_OK;
}

chasm_status chasm_advect_history(chasm_advect_t h, double* out, int32_t max_steps, int32_t* n_out)
{
    if (!h || !n_out || (max_steps > 0 && !out)) return fail(CHASM_EINVAL, "NULL argument");
    if (max_steps < 0) return fail(CHASM_EINVAL, "max_steps must be >= 0");
    if (!h->hist) return fail(CHASM_EINVAL, "handle was created without CHASM_FLAG_REDUCE_EACH_STEP");
    if (h->poisoned) return fail(CHASM_ESTATE, "handle is poisoned by an earlier device failure");
    int count = 0;
    hipError_t e = hipMemcpyAsync(&count, h->counter, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "history counter read");
    const int avail = std::min(count, h->hist_cap);
    const int n = std::min(avail, (int)max_steps);
    const size_t row = (size_t)h->desc.nbatch * NRED;
    std::vector<double> ring((size_t)h->hist_cap * row);
    e = hipMemcpy(ring.data(), h->hist, ring.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e, "history copy");
    // oldest kept entry is step count - avail; return the first n of the kept ones
    for (int i = 0; i < n; ++i) {
        const int step = count - avail + i;
        std::memcpy(out + (size_t)i * row, ring.data() + (size_t)(step % h->hist_cap) * row, row * sizeof(double));
    }
    *n_out = n;
    return CHASM_OK;
}

chasm_status chasm_advect_schedule(chasm_advect_t h, int32_t* schedule)
{
    if (!h || !schedule) return fail(CHASM_EINVAL, "NULL argument");
    *schedule = h->schedule;
    return CHASM_OK;
}

chasm_status chasm_advect_destroy(chasm_advect_t h)
{
    if (!h) return CHASM_OK;
    hipError_t e = hipSuccess;
    if (h->stream || h->tables) e = hipStreamSynchronize(h->stream);
    if (h->gexec) hipGraphExecDestroy(h->gexec);
    if (h->graph) hipGraphDestroy(h->graph);
    if (h->gexec2) hipGraphExecDestroy(h->gexec2);
    if (h->graph2) hipGraphDestroy(h->graph2);
    if (h->gexeck) hipGraphExecDestroy(h->gexeck);
    if (h->graphk) hipGraphDestroy(h->graphk);
    if (h->gexec_r) hipGraphExecDestroy(h->gexec_r);
    if (h->graph_r) hipGraphDestroy(h->graph_r);
    for (int g = 0; g < SG_COUNT; ++g) {
        if (h->sgexec[g]) hipGraphExecDestroy(h->sgexec[g]);
        if (h->sgraph[g]) hipGraphDestroy(h->sgraph[g]);
    }
    if (h->stage) hipFree(h->stage);
    if (h->cap_stream) hipStreamDestroy(h->cap_stream);
    if (h->tables) hipFree(h->tables);
    if (h->partials) hipFree(h->partials);
    if (h->fold) hipFree(h->fold);
    if (h->marg_part) hipFree(h->marg_part);
    if (h->marg_out) hipFree(h->marg_out);
    if (h->last) hipFree(h->last);
    if (h->hist) hipFree(h->hist);
    if (h->counter) hipFree(h->counter);
    delete h;
    if (e != hipSuccess) return fail(CHASM_EDEVICE, std::string("destroy: ") + hipGetErrorString(e));
    return CHASM_OK;
}

}  // extern "C"

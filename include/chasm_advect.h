/*
 * chasm_advect.h -- C ABI of the MI355X (gfx950) characteristic step of the CHASM
 * scheme for the 6-D Wigner equation.
 *
 * Paper: Y. Xiong, Y. Zhang, S. Shao, "A characteristic-spectral-mixed scheme for
 * six-dimensional Wigner-Coulomb dynamics", arXiv:2205.02380.
 *
 * The library advances a phase-space function f(x, k) along the characteristic flow
 * A_tau(x, k) = (x - k dt, k) of the free-streaming Wigner equation (Sec. 2.2,
 * eq. 2.6, hbar = m = 1):  f_new(x, k) = f(x - k dt, k).  The shift is interpolated
 * with patch-local cubic B-splines (Sec. 3.1): every patch of M cells solves its own
 * spline coefficients, closed by the perfectly matched boundary condition (PMBC,
 * eqs. 3.4-3.5) whose stencils reach g nodes into the neighbouring patches, and
 * the patch whose cells contain a departure point evaluates it (Sec. 3.1.3).  The
 * 3-D shift is applied as three successive axis sweeps x1, x2, x3 (the tensor-product
 * spline of Sec. 3.2, eqs. 3.11-3.12).
 *
 * No C++ types and no exceptions cross this boundary.  All device pointers are plain
 * HIP device addresses; hip_stream is a hipStream_t passed as void* (NULL = the
 * default stream).
 *
 * Field layout (caller-owned device memory, contiguous):
 *   f[b][k3][k2][k1][x3][x2][x1], x1 fastest, b < nbatch independent fields of the
 *   same grid.  Element type float (CHASM_F32) or double (CHASM_F64).
 * Grids are half-open: x_{d,i} = x_lo[d] + i*h_d, h_d = (x_hi[d]-x_lo[d])/nx[d],
 *   k_{d,i} = k_lo[d] + i*hk_d, hk_d = (k_hi[d]-k_lo[d])/nk[d].
 * Patches along an axis of N nodes: p = ceil((N-1)/M) patches of M cells sharing end
 *   nodes (eq. 3.1), the last one possibly shorter.
 *
 * Errors: every call returns a chasm_status; on failure chasm_advect_last_error()
 * returns a message for the calling thread.  A handle whose device work failed is
 * poisoned and returns CHASM_ESTATE until destroyed.  Handles are not thread-safe:
 * one owning thread per handle.
 */
#ifndef CHASM_ADVECT_H
#define CHASM_ADVECT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chasm_advect_s* chasm_advect_t;   /* opaque handle */

typedef enum {
    CHASM_OK = 0,
    CHASM_EINVAL = -1,        /* invalid argument or descriptor */
    CHASM_ENOMEM = -2,        /* device or host allocation failed */
    CHASM_EDEVICE = -3,       /* a HIP call or kernel launch failed */
    CHASM_ESTATE = -4,        /* handle poisoned by an earlier device failure */
    CHASM_EUNSUPPORTED = -5   /* valid, but beyond a resource limit of the kernels (or a
                                 schedule the shape's kernels do not provide) */
} chasm_status;

typedef enum { CHASM_F32 = 0, CHASM_F64 = 1 } chasm_dtype;

typedef enum {
    /* The paper's closure: interface slopes from rows of the inverse of the
     * natural-BC global spline matrix, truncated to |j - I| <= ghost (eqs. 3.3-3.5);
     * ghost splines beyond the outer line ends carry coefficient 0 (Sec. 3.1.3). */
    CHASM_CLOSURE_PMBC = 0,
    /* Variant not in the paper: the same rows plus the minimum-norm correction that
     * makes them exact for cubic data, and outer ghost coefficients extrapolated by a
     * zero fourth difference, so cubic polynomials in x are advected exactly.
     * Needs ghost >= 3. */
    CHASM_CLOSURE_POLY3 = 1,
    /* The paper's PMBC with the Neumann global condition instead of the natural one:
     * rows of the inverse of the global matrix with the Hermite boundary rows of
     * eq. 2.13 and zero end slopes, truncated to |j - I| <= ghost; the slopes at both
     * line ends are 0. */
    CHASM_CLOSURE_NEUMANN = 2,
    /* The paper's PMBC with the Hermite global condition of eq. 2.13 and given end
     * slopes: s'(x_lo) = slope_lo[d], s'(x_last) = slope_hi[d] on every line along axis
     * d (the Neumann closure is the case of zero slopes).  Interface slopes come from
     * the rows of the inverse of that global matrix: the data columns truncated to
     * |j - I| <= ghost, and the columns of the two given slopes kept for interfaces
     * within ghost of their end (reading in the design notes).  Runs on the
     * runtime-shape kernels. */
    CHASM_CLOSURE_HERMITE = 3
} chasm_closure;

typedef enum {
    CHASM_SCHED_AUTO = 0,     /* CUBE when the x-cube fits in LDS, else SLAB; PLAIN on the
                                 runtime-shape kernels */
    CHASM_SCHED_CUBE = 1,     /* one launch per step, all three sweeps in LDS */
    CHASM_SCHED_SLAB = 2,     /* two launches per step: x1+x2 on x3-slabs, then x3 */
    CHASM_SCHED_PLAIN = 3     /* three launches per step, one per axis */
} chasm_schedule;

enum {
    CHASM_FLAG_REDUCE_EACH_STEP = 1u << 0,   /* record FP64 diagnostics after every step */
    CHASM_FLAG_GRAPH = 1u << 1,              /* replay steps as captured HIP graphs (one graph
                                                per step, and one per 8 steps for long calls) */
    /* Allocate a second field of the same shape and dtype (the stage field, one more
     * field of device memory, owned by the handle) and run the sweeps out of place:
     * SLAB and PLAIN read f in their first launch and write the stage field, and write
     * f back in their last launch, so every step ends in f; CUBE runs the steps of one
     * chasm_advect_step call in pairs (f -> stage -> f) and an odd last step in place.
     * The arithmetic is unchanged (results are bitwise equal to in place); HBM serves a
     * read stream and a write stream to different addresses faster than read-modify-
     * write traffic on one buffer.  chasm_advect_step_many steps CUBE handles in place. */
    CHASM_FLAG_OUT_OF_PLACE = 1u << 2,
    /* Use the runtime-shape kernels even where compiled kernels exist for the shape
     * (every descriptor the compiled kernels do not cover uses them anyway): one launch
     * per axis sweep with the tables read from device memory, the PLAIN schedule. */
    CHASM_FLAG_RUNTIME_SHAPE = 1u << 3,
    /* Bits 4-5: launch-shape variant of the compiled SLAB and PLAIN passes (the
     * autotuner's tile-shape axis), CHASM_FLAG_TILE(t) for t = 0 (default), 1 (twice
     * the x3-slabs per slab block, 128 lines per pencil block) or 2 (default slab block,
     * 384 or 512 lines per pencil block).  Variants 1 and 2 exist for the FP32 shapes
     * with nx = 48 or 64 and need the SLAB or PLAIN schedule named explicitly (else
     * CHASM_EUNSUPPORTED).  The arithmetic does not depend on the variant: results are
     * bitwise equal. */
    CHASM_FLAG_TILE_SHIFT = 4,
    CHASM_FLAG_TILE_MASK = 3u << 4,
    /* Observe every call: the x3 sweep that ends the last step of each
     * chasm_advect_step call with nsteps >= 1 also forms, in its epilogue, the FP64
     * item rows of the observables of Sec. 5 (W1, W2, W3, P; see
     * chasm_advect_marginals), and a short pass sums them; chasm_advect_observables
     * returns them.  That last step runs its sweeps in the order x1, x2, x3 as three
     * launches (SLAB and CUBE handles included); on a SLAB handle, whose steps
     * alternate the sweep order, the field it leaves can differ from an unobserved run
     * in the last bits.  The observables are bitwise equal to chasm_advect_marginals of
     * the stored field.  The handle allocates the item rows
     * (nbatch * nk1 nk2 nk3 * (nx1 nx2 + ceil(nx1 nx2 / 64) nx3) doubles) at create.
     * A handle with this flag is stepped on its own by chasm_advect_step_many. */
    CHASM_FLAG_OBSERVE = 1u << 6
};
#define CHASM_FLAG_TILE(t) ((uint32_t)(t) << CHASM_FLAG_TILE_SHIFT)

typedef struct {
    int32_t nx[3];            /* x nodes per axis (>= 2); grids with equal nx and patch on the
                                 three axes and a compiled (nx, patch, ghost) run the compiled
                                 kernels, every other grid the runtime-shape kernels */
    int32_t nk[3];            /* k nodes per axis (>= 1) */
    double x_lo[3], x_hi[3];  /* half-open x extents */
    double k_lo[3], k_hi[3];  /* half-open k extents */
    int32_t patch[3];         /* cells per patch M_d (>= 1) */
    int32_t ghost;            /* PMBC stencil half-width g = n_nb (>= 1; >= 3 for POLY3) */
    double dt;                /* time step (hbar = m = 1) */
    int32_t dtype;            /* chasm_dtype */
    int32_t closure;          /* chasm_closure */
    int32_t nbatch;           /* independent fields of this grid, leading dimension b (>= 1) */
    uint32_t flags;           /* CHASM_FLAG_* */
    int32_t schedule;         /* chasm_schedule */
    int32_t history_cap;      /* steps of diagnostics kept with REDUCE_EACH_STEP (0: 1024) */
    double slope_lo[3], slope_hi[3];   /* end slopes of CHASM_CLOSURE_HERMITE (else ignored) */
} chasm_advect_desc;

/* Create a handle that advances the caller's field f_dev in place.
 * Builds the per-axis FP64 tables on the host (interface stencils, patch factors,
 * per-k shift weights; eqs. 3.4-3.8), copies them to the device, and picks kernels.
 * f_dev: device pointer, 16-byte aligned, nbatch*prod(nk)*prod(nx) elements of the
 *   dtype; owned by the caller, never freed by the library, must outlive the handle.
 * hip_stream: stream all work of this handle is issued on.
 * Errors: EINVAL (bad descriptor or pointer), EUNSUPPORTED (beyond a resource limit:
 *   a line too long for the LDS tiles, a launch grid beyond 2^31 blocks; or CUBE/SLAB
 *   asked of the runtime-shape kernels), ENOMEM, EDEVICE. */
chasm_status chasm_advect_create(const chasm_advect_desc* desc, void* f_dev, void* hip_stream,
                                 chasm_advect_t* out);

/* Advance the field by nsteps steps of dt (each step: x1, x2, x3 sweeps, Sec. 3.2).
 * Asynchronous on the handle's stream.  nsteps == 0 is a no-op; nsteps < 0 -> EINVAL. */
chasm_status chasm_advect_step(chasm_advect_t h, int32_t nsteps);

/* FP64 diagnostics of the current field (Sec. 5: grid sums times the cell volume
 * V = prod h_d * prod hk_d, summed over the batch): mass = V sum f; l2 = V sum f^2
 * (nullable); moments6 = V sum x_d f (d = 1..3) then V sum k_d f (nullable).
 * Synchronises the handle's stream. */
chasm_status chasm_advect_mass(chasm_advect_t h, double* mass, double* l2, double* moments6);

/* Per-batch-member diagnostics of the current field: out[b*8 + i], i = mass, l2,
 * sum x1 f, x2, x3, k1, k2, k3 (all times V).  out holds nbatch*8 doubles (host).
 * Synchronises the handle's stream. */
chasm_status chasm_advect_diagnostics(chasm_advect_t h, double* out);

/* Allocation-free form of chasm_advect_diagnostics, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  No handle: desc describes the field f_dev (same rules as
 * chasm_advect_create; the FP64 results are those chasm_advect_diagnostics returns for
 * a handle over f_dev, bitwise).  out_dev: caller-owned DEVICE memory of nbatch*8
 * doubles, written as out_dev[b*8 + i] (i = mass, l2, x1, x2, x3, k1, k2, k3, all times
 * V).  Asynchronous on hip_stream; nothing is allocated and nothing is copied to the
 * host.  The partial sums live in a fixed 16 MiB device workspace of the library (one
 * per GPU, held until the process ends): fields whose nbatch*prod(nk) partial rows
 * (64 bytes each, plus 16 KiB per batch member) exceed it return CHASM_EINVAL.  Every
 * call on a GPU shares that GPU's workspace, so calls that overlap on one GPU (other
 * streams or threads) race; serialise them.
 * Errors: EINVAL (bad descriptor, pointer or size), EUNSUPPORTED, EDEVICE. */
chasm_status chasm_advect_diagnostics_noalloc(const chasm_advect_desc* desc, const void* f_dev, void* hip_stream,
                                              double* out_dev);

/* The visualisation observables of Sec. 5 for each batch member b, in FP64 (host
 * arrays; any may be NULL to skip it):
 *   w1[b][k1][x1] = W_1(x1, k1) = integral of f over x2, x3, k2, k3  (nbatch*nk[0]*nx[0])
 *   w2[b][k2][x2], w3[b][k3][x3] likewise                              (nbatch*nk[d]*nx[d])
 *   p12[b][x2][x1] = P(x1, x2) = integral of f over x3 and k           (nbatch*nx[1]*nx[0])
 * Integrals are cell sums times the spacings of the integrated variables (the
 * paper's "average over the grid" convention, as for the mass).  The field is read
 * once; the first call allocates nbatch*nk1*nk2*nk3*(3N + N^2) doubles of device
 * workspace, kept until destroy.  Synchronises the handle's stream. */
chasm_status chasm_advect_marginals(chasm_advect_t h, double* w1, double* w2, double* w3, double* p12);

/* The observables of the field left by the last chasm_advect_step call (nsteps >= 1)
 * of a handle created with CHASM_FLAG_OBSERVE, formed in that call's last x3 sweep
 * (Sec. 5 observables as fused FP64 reductions).  Same layout and values as
 * chasm_advect_marginals would give on that field, bitwise.  Host pointers, each
 * nullable; synchronises the stream.  A chasm_advect_marginals call on the handle
 * reuses the same buffers and replaces them.  CHASM_EINVAL without the flag, before
 * the first observed call, or after a marginals call until the next observed call. */
chasm_status chasm_advect_observables(chasm_advect_t h, double* w1, double* w2, double* w3, double* p12);

/* Diagnostics recorded by CHASM_FLAG_REDUCE_EACH_STEP, oldest first:
 * out[s*nbatch*8 + b*8 + i] for s < *n_out (at most max_steps, host memory).
 * Synchronises the handle's stream. */
chasm_status chasm_advect_history(chasm_advect_t h, double* out, int32_t max_steps, int32_t* n_out);

/* Advance several handles by nsteps[i] steps each.  Handles with the same dtype,
 * grid shape, patch and ghost width share one launch per sweep (their items are
 * concatenated in a device work list); all handles must use the same stream.
 * Asynchronous. */
chasm_status chasm_advect_step_many(const chasm_advect_t* hs, int32_t n, const int32_t* nsteps);

/* Device bytes the library allocates for a handle with this descriptor (tables,
 * partials, history), not counting the caller's field. */
chasm_status chasm_advect_workspace_bytes(const chasm_advect_desc* desc, size_t* bytes);

/* Schedule actually used by a handle (after AUTO resolution). */
chasm_status chasm_advect_schedule(chasm_advect_t h, int32_t* schedule);

/* Release everything the library allocated for h.  Synchronises its stream.
 * NULL is a no-op. */
chasm_status chasm_advect_destroy(chasm_advect_t h);

/* Message of the last failed call on this thread ("" if none). */
const char* chasm_advect_last_error(void);

/* Library version string. */
const char* chasm_advect_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHASM_ADVECT_H */

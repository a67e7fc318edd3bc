/*
 * chasm_theta.h -- C ABI of the truncated-kernel evaluation of the Coulomb
 * pseudo-differential operator Theta_V on MI355X (gfx950).
 *
 * Paper: Y. Xiong, Y. Zhang, S. Shao, "A characteristic-spectral-mixed scheme for
 * six-dimensional Wigner-Coulomb dynamics", arXiv:2205.02380, Sec. 4.
 *
 * For the attractive potential V(x) = -sum_a z_a / |x - x_a| (atomic units, Sec. 2.1)
 * the operator of eq. 2.4 is, per nucleus, a twisted convolution in k with the
 * singular kernel |k|^-2.  The truncated kernel method (Sec. 4.1) replaces it by the
 * discrete convolution of eq. 4.8 with the tensor T of eq. 4.9 (threefold dual grid
 * of eq. 4.10, kernel truncated at D = diam Omega), applied to the modulated data
 * e^{-2i (x - x_a).k} f and demodulated as in eq. 4.6:
 *   out(x, k_p) = sum_a z_a Theta^T_a[f](x, k_p).
 * The k-box Omega is the half-open grid box of side nk_d * hk_d; D is its diameter.
 * The library builds T and its transform on the host in FP64 once per handle and
 * evaluates the convolutions in FP64 on the device (FFT of period 2 nk per axis,
 * zero padded), whatever the storage type of the field.  For nk 8 and 16 one block
 * holds an x-point's whole transform in LDS; for nk 32 and 64 (and on request 16) the
 * staged form runs the transforms over batches of x-points with a complex FP64
 * intermediate of 2 nk^3 values per x-point in device memory (at most about 2 GiB per
 * handle, plus nk^3 doubles per x-point of the batch for more than one nucleus).
 *
 * Field layout: as in chasm_advect.h, f[b][k3][k2][k1][x3][x2][x1] (x1 fastest),
 * caller-owned contiguous device memory of float (CHASM_F32) or double (CHASM_F64).
 * Grids are half-open with the same conventions as chasm_advect.h.
 *
 * Status codes and the error message (chasm_advect_last_error) are shared with
 * chasm_advect.h.  Handles are not thread-safe: one owning thread per handle.
 */
#ifndef CHASM_THETA_H
#define CHASM_THETA_H

#include <stddef.h>
#include <stdint.h>

#include "chasm_advect.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CHASM_THETA_MAX_NUCLEI 4

typedef struct chasm_theta_s* chasm_theta_t;   /* opaque handle */

/* Descriptor flags. */
#define CHASM_THETA_FLAG_STAGED 1u   /* use the staged form (below) also where the one-block
                                        form exists (nk 16) */

typedef struct {
    int32_t nx[3], nk[3];          /* grid nodes per axis; nk[0] = nk[1] = nk[2] in {8, 16, 32, 64} */
    double x_lo[3], x_hi[3];       /* half-open x box */
    double k_lo[3], k_hi[3];       /* half-open k box (Omega) */
    int32_t nnuc;                  /* 1 .. CHASM_THETA_MAX_NUCLEI */
    double x_nuc[CHASM_THETA_MAX_NUCLEI][3];   /* nucleus positions x_a */
    double z_nuc[CHASM_THETA_MAX_NUCLEI];      /* charges z_a (1 for a proton) */
    int32_t dtype;                 /* chasm_dtype of the field and of the output */
    int32_t nbatch;                /* independent fields of this grid, leading dim b */
    uint32_t flags;                /* CHASM_THETA_FLAG_* */
} chasm_theta_desc;

/* Create a handle: validates the descriptor (CHASM_EINVAL; CHASM_EUNSUPPORTED for
 * an nk without kernels), builds T and its transform in FP64 on the host, uploads the
 * transform and allocates one field-sized workspace (x-major copy) and, for the staged
 * form, its batch intermediate.  hip_stream is a
 * hipStream_t (NULL = default stream) used by every later call. */
chasm_status chasm_theta_create(const chasm_theta_desc* desc, void* hip_stream, chasm_theta_t* out);

/* out = Theta^T[f] (eq. 4.6 summed over the nuclei), asynchronously on the handle's
 * stream.  f and out are device pointers to fields of the descriptor's shape and
 * dtype; out may equal f (f is consumed before out is written).  Neither is retained
 * after the call. */
chasm_status chasm_theta_apply(chasm_theta_t h, const void* f_dev, void* out_dev);

/* Device bytes a handle of this descriptor allocates (workspace + tables). */
chasm_status chasm_theta_workspace_bytes(const chasm_theta_desc* desc, size_t* bytes);

/* Host-only: the tensor T_p of eq. 4.9 for p_d = -(nk_d - 1) .. nk_d - 1 as the
 * library builds it, written to t_host as [p3][p2][p1] ((2 nk - 1)^3 doubles). */
chasm_status chasm_theta_tensor(const chasm_theta_desc* desc, double* t_host);

/* Release a handle (NULL is a no-op). */
chasm_status chasm_theta_destroy(chasm_theta_t h);

#ifdef __cplusplus
}
#endif

#endif /* CHASM_THETA_H */

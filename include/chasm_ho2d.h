/*
 * chasm_ho2d.h -- C ABI of the 2-D (x, k) harmonic-oscillator Wigner workload on MI355X
 * (gfx950): the CHASM scheme with a local potential.
 *
 * Paper: Y. Xiong, Y. Zhang, S. Shao, "A characteristic-spectral-mixed scheme for
 * six-dimensional Wigner-Coulomb dynamics", arXiv:2205.02380, Sec. 5.1.
 *
 * For V(x) = omega x^2 / 2 (m = hbar = 1) the pseudo-differential operator reduces to a
 * first-order derivative, Theta[f] = omega x d_k f (eq. 5.1).  The library advances
 * f(x, k) by LPC1 (Sec. 2.2): the characteristic step in x of every k-line with the
 * patched cubic spline of Sec. 3 (PMBC, natural closure, patches of `patch` cells,
 * stencil half-width `ghost`), and Theta from the spectral derivative in k on the
 * periodic k-grid (F^-1 diag(i xi) F, Nyquist mode set to zero): by FFT when nk is a
 * power of two in 64..1024, else as the product with the circulant differentiation
 * matrix.  Everything is FP64.
 *
 * Inflow: the paper's run of this example to T = 10 (dx = 0.1, dk = 0.025, tau = 2e-5)
 * is stable with zero inflow; evaluating inflow departure points from the ghost-extended
 * spline lets a boundary mode grow from rounding (about e^4 per unit time at x = 12)
 * and overtake the solution after t ~ 7 on that grid.
 *
 * Field: f[k][x] (x fastest), nk * nx doubles of caller-owned device memory, advanced
 * in place.  x_i = x_lo + i hx (i < nx); k_i = k_lo + i hk (i < nk, nk even).
 * Status codes and chasm_advect_last_error() are shared with chasm_advect.h.
 */
#ifndef CHASM_HO2D_H
#define CHASM_HO2D_H

#include <stdint.h>

#include "chasm_advect.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chasm_ho2d_s* chasm_ho2d_t;   /* opaque handle */

typedef struct {
    int32_t nx;            /* x nodes, 2 .. 1024 */
    double x_lo, hx;
    int32_t nk;            /* k nodes, even, 2 .. 4096 */
    double k_lo, hk;
    int32_t patch;         /* cells per patch M (the last patch may be shorter) */
    int32_t ghost;         /* PMBC stencil half-width g >= 1 */
    double omega;          /* V = omega x^2 / 2 */
    double tau;            /* time step */
    int32_t inflow;        /* departure points outside [x_0, x_{nx-1}]: 0 give 0 (zero inflow),
                              1 are evaluated by the outer patch with its ghost coefficients
                              (the convention of chasm_advect.h) */
} chasm_ho2d_desc;

/* Validate (CHASM_EINVAL), build the FP64 tables on the host (PMBC stencils, patch
 * inverses, per-k shift weights, the k-differentiation matrix), allocate six fields of
 * state.  f_dev is the caller's field; hip_stream a hipStream_t (NULL = default). */
chasm_status chasm_ho2d_create(const chasm_ho2d_desc* desc, void* f_dev, void* hip_stream, chasm_ho2d_t* out);

/* nsteps LPC1 steps on the field, in place, asynchronously (negative: CHASM_EINVAL). */
chasm_status chasm_ho2d_step(chasm_ho2d_t h, int32_t nsteps);

/* Release (NULL is a no-op). */
chasm_status chasm_ho2d_destroy(chasm_ho2d_t h);

#ifdef __cplusplus
}
#endif

#endif /* CHASM_HO2D_H */

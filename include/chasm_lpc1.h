/*
 * chasm_lpc1.h -- C ABI of the one-stage Lawson predictor-corrector (LPC1) time step
 * of the Wigner-Coulomb equation on MI355X (gfx950): the characteristic step of
 * chasm_advect.h combined with the truncated-kernel Theta_V of chasm_theta.h.
 *
 * Paper: Y. Xiong, Y. Zhang, S. Shao, "A characteristic-spectral-mixed scheme for
 * six-dimensional Wigner-Coulomb dynamics", arXiv:2205.02380, Sec. 2.2 (LPC1).
 *
 * With A the characteristic shift g -> g o A_tau (chasm_advect_step, one step of dt =
 * tau) and Theta the truncated-kernel operator (chasm_theta_apply), one step is
 *   predictor  f~      = A f^n + tau A Theta[f^n]
 *   corrector  f^{n+1} = A f^n + tau/2 Theta[f~] + tau/2 A Theta[f^n].
 * A is applied once per step to f^n and to Theta[f^n] (one advection handle for each);
 * Theta is evaluated twice per step.
 *
 * The field (caller-owned, layout and dtype of chasm_advect.h, nbatch 1) is advanced
 * in place and is itself the state: the library keeps Theta[f^n] and the predictor in
 * two fields of its own, and no step copies the field.  If a step fails the handle is
 * poisoned and the field may hold a partly updated step.  Status codes and chasm_advect_last_error() are
 * shared with chasm_advect.h.  Handles are not thread-safe.
 */
#ifndef CHASM_LPC1_H
#define CHASM_LPC1_H

#include <stdint.h>

#include "chasm_advect.h"
#include "chasm_theta.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chasm_lpc1_s* chasm_lpc1_t;   /* opaque handle */

/* adv describes the grid, splines and tau (= adv->dt); its nbatch must be 1 and its
 * flags 0.  th must describe the same grid and dtype with nbatch 1.  f_dev is the
 * caller's field; it must stay allocated until chasm_lpc1_destroy.  Allocates two
 * fields plus the workspaces of the operators (two advection handles, one Theta).  CHASM_EINVAL on mismatched
 * descriptors; the errors of chasm_advect_create / chasm_theta_create otherwise. */
chasm_status chasm_lpc1_create(const chasm_advect_desc* adv, const chasm_theta_desc* th, void* f_dev,
                               void* hip_stream, chasm_lpc1_t* out);

/* Advance the field by nsteps LPC1 steps (asynchronous on the handle's stream;
 * nsteps = 0 is a no-op, negative is CHASM_EINVAL). */
chasm_status chasm_lpc1_step(chasm_lpc1_t h, int32_t nsteps);

/* Release a handle and its operators (NULL is a no-op). */
chasm_status chasm_lpc1_destroy(chasm_lpc1_t h);

#ifdef __cplusplus
}
#endif

#endif /* CHASM_LPC1_H */

/*
 * enkf_l96.h -- Lorenz-96 ensemble forecast on one MI355X (gfx950), the model
 * step of the cycling filter of the Lorenz-96 experiments (Section 4).
 *
 *   dx_i/dt = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F,   i cyclic (eq. Lorenz96),
 * advanced by classical fourth-order Runge-Kutta steps of length dt (the
 * experiments use F = 8; the workloads here use dt = 0.05).
 *
 * Conventions as in enkf_sm.h: column-major FP64 device arrays, stream
 * ordered, enkf_status returns, argument errors found on the host.
 */
#ifndef ENKF_L96_H
#define ENKF_L96_H

#include <stdint.h>

#include "enkf_sm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ENKF_L96_MAX_STATE 8192   /* n_state <= 8192 (one member's state in LDS) */

/*
 * Advance every column of X (n_state x m, FP64, leading dimension ldx >=
 * n_state, DEVICE) by nsteps RK4 steps, in place. One workgroup per member.
 * 4 <= n_state <= ENKF_L96_MAX_STATE, m >= 0, nsteps >= 0, dt and F finite;
 * otherwise ENKF_ERR_INVALID_ARG (n_state above the maximum:
 * ENKF_ERR_NOT_SUPPORTED). Allocates nothing.
 */
enkf_status enkf_l96_forecast(int64_t n_state, int32_t m, double* X, int64_t ldx, int32_t nsteps, double F, double dt,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ENKF_L96_H */

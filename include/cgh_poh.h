/* cgh_poh.h -- C ABI of the phase-only hologram (POH) conversion of the
 * paper's complex hologram (Sec. 3.3), gfx950.
 *
 * Smooth POH: double-phase amplitude coding.  The printed formula assigns the
 * amplitude itself to the even cells; it is read as the double-phase coding of
 * Hsueh and Sawchuk (1978) used by Maimone et al. (2017): per colour channel
 * A_n = |H| / max |H| (0 when H = 0 everywhere), phi = arg H, and the phase is
 * phi + arccos(A_n) where row + column is even, phi - arccos(A_n) where odd, so
 * that two neighbouring phasors average to A_n e^{j phi}.
 *
 * Random POH: a per-pixel phase phi_rand optimised jointly with the Gaussians
 * under L_extract = L_recon(I, T) + L_recon(I_rand, T) + l_comp ||I - I_rand||^2
 * + l_field ||U - U_rand||_{1,C} (the paper uses l_comp = 0.1, l_field = 0.01;
 * every norm is a mean over the L C H W elements, and the plane sum of the
 * paper becomes the corresponding average).  The library supplies the seed of
 * the two adjoint propagations (cgh_poh_extract_seed), the field
 * exp(j phi_rand) and the phase gradient; the propagations are cgh_propagate
 * and cgh_propagate_field_adjoint (cgh.h).
 *
 * All pointers are device pointers owned by the caller; every call only
 * enqueues work on `stream` and allocates nothing.  Argument errors return
 * CGH_ERR_INVALID_ARG before any launch.
 */
#ifndef CGH_POH_H
#define CGH_POH_H

#include <stddef.h>
#include <stdint.h>

#include "cgh.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Smooth POH phases of field ([C][H][W] complex) into phase ([C][H][W]).
 * amax: caller scratch of C floats (the per-channel maxima). */
cgh_status cgh_poh_dpac(const cgh_c64 *field, int32_t C, int32_t H, int32_t W, float *amax,
                        float *phase, void *stream);

/* field[i] = exp(j phase[i]), i < count. */
cgh_status cgh_poh_field(const float *phase, int64_t count, cgh_c64 *field, void *stream);

/* grad_phase[i] = dL/dphase[i] = Im(conj(exp(j phase[i])) g[i]) for
 * g = dL/dRe(H) + j dL/dIm(H) of H = exp(j phase). */
cgh_status cgh_poh_phase_grad(const float *phase, const cgh_c64 *grad_field, int64_t count,
                              float *grad_phase, void *stream);

/* Number of FP64 partial sums cgh_poh_extract_seed needs for `count` elements. */
int64_t cgh_poh_extract_partials(int64_t count);

/* L_extract for the propagated fields u (of the Gaussians' hologram) and
 * u_rand (of the random POH), both [L][C][H][W] complex, against target
 * ([L][C][H][W]) with optional focal masks ([L][H][W]; NULL: L_MSE terms).
 * Writes grad_u = dL/dRe(u) + j dL/dIm(u) and grad_u_rand likewise (the seeds
 * of cgh_propagate_field_adjoint), and loss[0] = L_extract (FP64; loss may be
 * NULL) through `partials` (>= cgh_poh_extract_partials doubles, caller
 * scratch); sums in a fixed order. */
cgh_status cgh_poh_extract_seed(const cgh_c64 *u, const cgh_c64 *u_rand, const float *target,
                                const float *mask, int32_t L, int32_t C, int32_t H, int32_t W,
                                float l_comp, float l_field, cgh_c64 *grad_u,
                                cgh_c64 *grad_u_rand, double *partials, double *loss,
                                void *stream);

#ifdef __cplusplus
}
#endif

#endif

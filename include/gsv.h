/*
 * gsv.h -- iterative Grover search on a dense statevector (AMD gfx950), the comparison
 * backend of the paper's Section III-A / Fig. 2: the state is re-fed through one Grover
 * gate G = D O (Eq. (3)) per iteration, with the oracle O = I - 2 sum_{x in W} |x><x| and the
 * diffusion D = 2|s><s| - I (Eq. (4)).
 *
 * Starting from |s> (Eq. (2)) every amplitude stays real, so the state is a real vector of
 * N = 2^n values: FP64 (GMPS_FP64) or FP32 (GMPS_MIXED: FP32 storage, FP64 reductions). One
 * iteration is one streaming pass over the vector, psi <- 2 mu - psi with mu the mean of
 * the oracle-flipped state, which also accumulates the sum the next mean needs, plus a
 * one-block kernel that flips the M marked amplitudes and corrects that sum.
 *
 * Conventions as in gmps.h: int status codes (GMPS_OK / GMPS_E_*), host pointers are read
 * during the call only, the device workspace is caller-owned and must outlive the handle,
 * work is enqueued on the given HIP stream (NULL: default stream); gsv_iterate is
 * asynchronous, calls returning host values synchronise. Bit i of an index x is qubit
 * n-1-i's value (most significant first), as in gmps.h.
 */
#ifndef GSV_H
#define GSV_H

#include <stddef.h>
#include <stdint.h>

#include "gmps.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsv_state gsv_state; /* opaque, library-owned */

/* Bytes of device workspace for an n-qubit state (1 <= n <= 34) in the given precision
 * (GMPS_FP64 or GMPS_MIXED; GMPS_FP32 is not a statevector precision and counts as invalid):
 * the vector (8 or 4 bytes per amplitude), the marked indices and a few reduction slots.
 * 0 on invalid input. */
size_t gsv_workspace_bytes(int32_t n, int32_t M, gmps_prec prec);

/* Creates a handle. marked: host [M], distinct, each < 2^n (copied). dev_workspace: device
 * memory of at least gsv_workspace_bytes() bytes, 256-byte aligned. The state is left
 * uninitialised: call gsv_init_uniform() next. Errors: GMPS_E_ARG, GMPS_E_WORKSPACE,
 * GMPS_E_UNSUPPORTED (no device), GMPS_E_HIP. */
int gsv_create(gsv_state** out, int32_t n, const uint64_t* marked, int32_t M, gmps_prec prec,
               void* dev_workspace, size_t ws_bytes, void* hip_stream);

/* Section II, Eq. (2): psi <- |s> (every amplitude 2^(-n/2)), k_done = 0. Asynchronous. */
int gsv_init_uniform(gsv_state* s);

/* Applies G = D O k >= 0 times (Eq. (3)); additive. Asynchronous. */
int gsv_iterate(gsv_state* s, int64_t k);

/* Eq. (6): sum_{x in W} psi(x)^2 / sum_x psi(x)^2 (the norm by a full FP64 reduction).
 * out_p: host [1]. Synchronises. */
int gsv_marked_prob(gsv_state* s, double* out_p);

/* psi(x) for cnt indices (each < 2^n). xs: host [cnt]; out: host [cnt]. Synchronises. */
int gsv_amplitudes(gsv_state* s, const uint64_t* xs, int64_t cnt, double* out);

/* Milliseconds of the last gsv_iterate() call on the handle's stream (HIP events around
 * its launches). Synchronises. */
int gsv_last_iterate_ms(gsv_state* s, double* ms);

/* Frees the handle (not the workspace). NULL is OK. */
int gsv_destroy(gsv_state* s);

#ifdef __cplusplus
}
#endif

#endif /* GSV_H */

/*
 * gmps.h -- batched iterative Grover search on matrix product states (AMD gfx950).
 *
 * The library simulates the paper's "iterative method" (Section III-A, Fig. 1(C)):
 * one Grover gate G = D O (Eq. (3)) is re-applied to a stored matrix product state
 * (Section III-B) k times. Each reflection -- the oracle I - 2|x><x| for every marked x
 * and the diffusion D = H^n (2|0><0| - I) H^n = 2|s><s| - I (Eq. (4)) -- is applied as a
 * bond-2 matrix product operator and followed by recompression: a QR
 * left-canonicalisation sweep and a truncated-SVD sweep (singular values below
 * trunc_tol * sigma_0 are dropped, at most chi_cap kept). The state is renormalised
 * after every iteration.
 *
 * Conventions shared by every call:
 *  - Status: every int-returning call returns GMPS_OK (0) or a negative GMPS_E_* code.
 *    Nothing throws across the ABI. gmps_strerror() names each code.
 *  - Bits: site i of the chain carries bit (n-1-i) of a basis index (most significant
 *    bit first). Marked indices, amplitude queries and sampled bitstrings all use it.
 *  - Memory: pointers documented as "host" are caller-owned host memory, read or
 *    written during the call only. The device workspace is caller-owned device memory
 *    (for example a torch uint8 tensor) that must outlive the batch handle. The batch
 *    handle itself is library-owned and freed by gmps_destroy().
 *  - Streams: device work is enqueued on the HIP stream given to gmps_create() (a
 *    hipStream_t passed as void*; NULL means the default stream). grover_iterate() and
 *    mps_init_uniform() are asynchronous; calls that return host values synchronise
 *    that stream first.
 *  - Threads: a handle is not thread-safe; distinct handles are independent.
 *  - Precision: GMPS_FP64 keeps site tensors and all arithmetic in complex128.
 *    GMPS_MIXED on the team kernel (the default) runs every arithmetic step in FP64 and
 *    stores the bulk of the chain in complex64. The rounding error of a stored isometry is
 *    split in two: the part inside the span of the stored vectors is folded into the FP64
 *    carry that moves on along the sweep (compensated rounding), and the rest is orthogonal
 *    to every state whose support at that bond lies in that span, as the Grover states'
 *    supports do. The sites within ceil(log2(M+1)) of either end, where a bond can be
 *    smaller than that support, and the norm-carrying end site are kept in complex128 in
 *    edge slots of the workspace. On the lane-group kernel GMPS_MIXED instead runs the MPO
 *    application and the site contractions in complex64 and the factorisations in FP64 on
 *    up-converted tiles. Either way Schmidt components below trunc_tol (5e-7) of the
 *    largest are dropped. Accuracy of the team kernel's GMPS_MIXED, measured against the
 *    rotation angle (2k+1) theta: at n <= 29 the angle error stays near 1e-8. At n = 40,
 *    where the marked amplitudes start at ~2^-20, the angle drifts by ~2e-9 per iteration, far
 *    beyond 1e-6 in P over the full k: such runs need GMPS_FP64. Near the
 *    peak of P, in the one iteration where the unmarked component passes through a few
 *    1e-6, the mixed path's rotation angle (2k+1) theta can shift by up to about 2e-6 rad;
 *    P, flat there, moves by ~1e-12, but the shift stays with the state if it is iterated
 *    on past the peak.
 *    GMPS_FP32 (the all-single-precision simulation whose accuracy Section IV / Fig. 3
 *    examines) runs everything in complex64 / FP32, factorisations included, with results
 *    rounded to nearest; it exists on the lane-group kernel only (gmps_options.kernel 0 or
 *    1; 2 returns GMPS_E_UNSUPPORTED), so effective bond caps above 6 return
 *    GMPS_E_UNSUPPORTED; no warm starts unless jacobi_warm = 1; default trunc_tol 1e-6.
 *    Read-outs (marked_prob, amplitudes, sampling) accumulate in FP64 on every path.
 */
#ifndef GMPS_H
#define GMPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmps_batch gmps_batch; /* opaque, library-owned */

typedef enum { GMPS_FP64 = 0, GMPS_MIXED = 1, GMPS_FP32 = 2 } gmps_prec;

enum {
  GMPS_OK = 0,
  GMPS_E_ARG = -1,         /* invalid argument; nothing was enqueued               */
  GMPS_E_WORKSPACE = -2,   /* workspace NULL, misaligned (<256 B) or too small, or  *
                            * a request beyond sample_shots_noalloc's static array  */
  GMPS_E_HIP = -3,         /* a HIP runtime call failed                             */
  GMPS_E_UNSUPPORTED = -4, /* no tile class holds the bond cap, an option the chosen *
                            * kernel or precision lacks, or no device               */
  GMPS_E_NUMERIC = -5      /* some instance reports NaN/Inf or norm drift (see      *
                            * gmps_diagnostics); results were still written         */
};

/* Per-instance status bits reported by gmps_diagnostics(). */
enum {
  GMPS_ST_NAN = 1,   /* a non-finite value appeared in the chain               */
  GMPS_ST_DRIFT = 2, /* |norm - 1| before a renormalisation exceeded 1e-3     */
  GMPS_ST_TRUNC = 4  /* a truncation dropped more than 1e-8 of the weight     */
};

/* One independent search: n qubits (1..63), M marked items (1 <= M < 2^n) whose
 * indices are marked[marked_off .. marked_off+M-1] (distinct, < 2^n), and the bond cap
 * chi_cap >= 1. Every state the iteration passes through is a combination of |s> and the
 * M marked basis states, so its Schmidt rank at any cut is at most M+1: the library caps
 * each bond at min(chi_cap, M+1, 2^floor(n/2)), which drops only rounding noise when
 * chi_cap >= M+1 and truncates physical weight (reported by gmps_diagnostics) otherwise. */
typedef struct {
  int32_t n;
  int32_t M;
  int32_t chi_cap;
  int32_t reserved; /* must be 0 */
  int64_t marked_off;
} gmps_instance;

/* Optional knobs; pass NULL for defaults. Zero-initialise unused fields. */
typedef struct {
  double trunc_tol;     /* relative SVD cut; <= 0: 1e-12 (FP64) or 5e-7 (mixed)       */
  int32_t max_sweeps;   /* one-sided Jacobi sweep cap per SVD; <= 0: 16                */
  int32_t waves_per_cu; /* persistent-grid occupancy; <= 0: library plan              */
  int32_t use_graph;    /* 1 (default when 0): replay grover_iterate from a hipGraph;
                           -1: plain launches                                         */
  int32_t round_mode;   /* GMPS_MIXED only: how an FP64 result stored as complex64 is rounded.
                           0 (default): to nearest on the team kernel, stochastically on the
                           lane-group kernel; 1: stochastically (unbiased, so the rounding
                           errors of successive iterations do not add up coherently);
                           -1: to nearest                                                */
  int32_t jacobi_warm;  /* 1: each Jacobi SVD starts from the unitary it produced at the
                           same (reflection, site) one iteration earlier, which keeps the
                           bond bases continuous across iterations; -1: start from the
                           identity; 0 (default): on for GMPS_MIXED on the lane-group kernel
                           (complex64 contractions; it removes a systematic drift at M = 1
                           there), off everywhere else. Ignored by the pipelined sweeps.    */
  int32_t kernel;       /* iterate kernel: 1 = lane-group kernel (a tile row per lane, up to 8
                           instances per wave; bond caps up to 6, larger caps go to the team
                           kernel), 2 = team kernel (a tile column per lane slot, one instance per
                           team of 16-256 threads; bond caps up to 32), 0 = library choice
                           (the team kernel; the lane-group kernel for GMPS_FP32) */
  int32_t precontract;  /* 1: projector pre-contraction, a recompression variant of Section III-B
                           (team kernel and GMPS_FP64 only; with kernel = 1, another precision, or
                           an instance whose effective bond cap exceeds 17, gmps_create returns
                           GMPS_E_UNSUPPORTED). A reflection
                           c0 I + c1 sum_t |p_t><p_t| over product states p_t (Eqs. (3)-(4): the
                           marked basis states for O, |s> for D) maps psi to
                           c0 psi + c1 sum_t <p_t|psi> p_t, an MPS of bond chi + T built from
                           the site tensors and the overlaps <p_t|psi> (contracted in a pass
                           before the QR sweep; with pipelined sweeps during it, the term
                           columns carrying overlaps predicted from the previous reflection
                           until the last site rescales them to the measured ones), instead
                           of a bond-2 MPO per projector (bond 2 chi).
                           When the bond cap is lossless (chi_cap >= min(M+1, 2^floor(n/2)))
                           and M fits the tile class, O is one reflection with T = M, so an
                           iteration takes two QR+SVD sweeps instead of M+1; otherwise each
                           marked index is one reflection with T = 1. Same result up to
                           rounding. It is refused on GMPS_MIXED: with complex64 storage the exact
                           product terms meet bond spaces tilted by the rounding of the stored
                           sites, and the rotation angle drifts, faster with n (sequential
                           sweeps: up to 3e-10 per iteration at M = 4 on the 4096-instance
                           workload, and at n = 40, M = 16 truncations ran away; pipelined
                           sweeps: |dP| 1.7e-5 on that workload). 0 or -1 (default): one bond-2
                           MPO per projector, as in the paper. */
  int32_t pipeline;     /* 0 or 1 (default): the team classes with bond caps 2, 3, 5 and 8 run
                           the reflections (bond-2 MPO or pre-contracted) with alternating sweep
                           directions on two waves, the truncation sweep of each reflection and
                           the canonicalisation sweep of the next in lock step one site apart;
                           ignored on the lane-group kernel and in a batch where some bond cap
                           is below the exact rank (a lossy truncation depends on the sweep
                           order; such a batch keeps the sequential, right-to-left
                           truncations). -1: one wave per instance, each reflection's two
                           sweeps in turn                                                  */
} gmps_options;

/* Bytes of device workspace gmps_create() needs for this batch with either iterate kernel
 * (0 on invalid input): the site arena, the complex128 edge slots, per-instance tables, and
 * a 16 MiB staging region that read-outs and sampling pass through in chunks, so no call
 * after gmps_create() allocates device memory. inst: host [B]; marked offsets are not read. */
size_t gmps_workspace_bytes(const gmps_instance* inst, int32_t B, gmps_prec prec);

/* Creates a handle over B instances. inst: host [B]; marked: host, every instance's
 * marked indices at its marked_off; both are copied. dev_workspace: device memory of at
 * least gmps_workspace_bytes() bytes, 256-byte aligned. hip_stream: hipStream_t or NULL.
 * The chain is left uninitialised: call mps_init_uniform() next.
 * Errors: GMPS_E_ARG (bad instance, duplicate or out-of-range marked index, unknown
 * kernel or precision), GMPS_E_WORKSPACE, GMPS_E_UNSUPPORTED (no tile class holds the bond
 * cap; precontract without the team kernel, on another precision than GMPS_FP64 or with an
 * effective bond cap above 17; GMPS_FP32
 * with kernel = 2 or an effective bond cap above 6), GMPS_E_HIP. */
int gmps_create(gmps_batch** out, const gmps_instance* inst, int32_t B, const uint64_t* marked,
                gmps_prec prec, const gmps_options* opt, void* dev_workspace, size_t ws_bytes,
                void* hip_stream);

/* Section II, Eq. (2): every instance <- |s> = |+>^n (bond dimension 1), k_done = 0,
 * diagnostics cleared. Asynchronous. */
int mps_init_uniform(gmps_batch* b);

/* Section III-A (Fig. 1(C)): applies G = D O (Eq. (3)) k times to every instance, in one
 * persistent kernel launch. k: host, k_len == 1 (same k for all) or k_len == B
 * (per-instance, each >= 0). Additive: k_done += k. Asynchronous. */
int grover_iterate(gmps_batch* b, const int64_t* k, int32_t k_len);

/* The Common method (Section III-A, Fig. 1(B)): instead of re-applying G, the whole circuit of
 * k stacked Grover layers is built once, as a gate list, and simulated gate by gate. Each layer
 * holds the gates of Fig. 1(A) in order: per marked x, an X on every qubit where x has a 0 (qubit
 * 0 the most significant bit), the n-controlled Z, the same X gates; then the diffusion as H and X
 * on every qubit, the n-controlled Z, X and H on every qubit. (As gates the diffusion is
 * 2|s><s| - I up to a sign, so a layer is -G and k layers give (-1)^k G^k |s>.) The initial H
 * layer is mps_init_uniform's. Every n-controlled Z is applied to the MPS as its exact bond-2 MPO
 * I - 2|1..1><1..1| with the QR and truncated-SVD sweeps of a reflection, the state renormalised
 * after it; the single-qubit gates between two of them act on the sites' physical index as the
 * QR sweep stages them (the gates on one qubit multiplied first), and those after the last one
 * act on the sites in place. The gate list lives in device memory that the caller owns: one
 * 32-bit word per gate (type in bits 8-15: 0 = H, 1 = X, 2 = n-controlled Z; qubit in bits 0-7).
 * FP64 and the team kernel only, bond caps up to 17, n >= 2.
 *
 * gmps_circuit_bytes: bytes of the gate lists of k layers for every instance (k: host, k_len == 1
 * or B, each >= 0; inst and marked as for gmps_create); 0 on invalid input. */
size_t gmps_circuit_bytes(const gmps_instance* inst, int32_t B, const uint64_t* marked, const int64_t* k,
                          int32_t k_len);

/* Builds every instance's k-layer gate list on the host and copies it into dev_gates (device,
 * at least gmps_circuit_bytes() bytes, 4-byte aligned, owned by the caller and read by
 * grover_circuit_run until the next build). Synchronises. Errors: GMPS_E_ARG, GMPS_E_WORKSPACE
 * (buffer too small or misaligned), GMPS_E_UNSUPPORTED (GMPS_MIXED, the lane-group kernel, an
 * instance with n < 2 or an effective bond cap above 17), GMPS_E_HIP. */
int gmps_circuit_build(gmps_batch* b, const int64_t* k, int32_t k_len, void* dev_gates, size_t bytes);

/* Runs the built circuits on the current chains (normally |s> from mps_init_uniform): one
 * launch of the sequential team kernels; k_done grows by each circuit's k. Asynchronous;
 * gmps_last_iterate_ms times it. Errors: GMPS_E_ARG (no circuit built), GMPS_E_HIP. */
int grover_circuit_run(gmps_batch* b);

/* grover_iterate and then perfect sampling of every instance's final state in the same graph
 * launch (a hit-counter fill kernel, the class kernels, the sampling kernel), for runs that
 * need the hit counts only. The draws are sample_shots' (same Philox stream, seed and shot
 * numbering), so out_hits equals sample_shots' out_hits after grover_iterate. shots: host,
 * shots_len == 1 or B (each >= 0); the shot offsets pass through the workspace's staging region.
 * out_hits: host [B] (may be NULL). gmps_last_iterate_ms then covers the sampling too.
 * Synchronises. Errors: GMPS_E_ARG, GMPS_E_WORKSPACE (B + 1 offsets beyond the staging
 * region), GMPS_E_HIP. */
int grover_iterate_sample(gmps_batch* b, const int64_t* k, int32_t k_len, const int64_t* shots, int32_t shots_len,
                          uint64_t seed, int64_t* out_hits);

/* Eq. (6): out_p[i] = sum_{x in W_i} |<x|psi_i>|^2 / <psi_i|psi_i>, accumulated in FP64.
 * out_p: host [B]. Synchronises. Returns GMPS_E_NUMERIC if any status bit is set. */
int marked_prob(gmps_batch* b, double* out_p);

/* Section IV (shots): perfect sampling of each instance's final state, site by site on
 * the right-canonical chain. shots: host, shots_len == 1 or B (each >= 0). The uniform for
 * (instance i, shot j, site t) is word t%4 of Philox4x64-10(counter = (j, t/4, 0, 0),
 * key = (seed, i)) as (word >> 11) * 2^-53; the site takes bit 0 iff u < p(0 | prefix).
 * out_bits: host [sum shots], instance-major; out_hits: host [B], the number of shots
 * that landed in W_i (either may be NULL). Synchronises. */
int sample_shots(gmps_batch* b, const int64_t* shots, int32_t shots_len, uint64_t seed,
                 uint64_t* out_bits, int64_t* out_hits);

/* sample_shots for callers that cannot allocate device memory or pass a staging buffer
 * (code under stream capture, tight serving loops, harnesses that forbid allocation). Same
 * arguments, results (bit for bit) and errors as sample_shots, but the hit counters, shot
 * offsets and bitstrings live in a static array of GMPS_NOALLOC_SCRATCH_BYTES that the library
 * holds in each GPU's memory from the first gmps_create() on that GPU until the process ends;
 * the call allocates nothing and uses no part of the workspace but the chain. Every call on a
 * GPU shares that GPU's array and leaves its contents behind: calls that overlap on one GPU
 * (other threads, other streams, other handles) race, so the caller serialises them.
 * Limits: 8*B bytes of counters plus 4.25 KiB of offsets plus 8 bytes per shot of one
 * instance must fit the array; a larger request returns GMPS_E_WORKSPACE before anything is
 * enqueued (instances are sampled in chunks, so only one instance's shots count).
 * GMPS_E_HIP if the array's device address could not be looked up. */
#define GMPS_NOALLOC_SCRATCH_BYTES (16u << 20)
int sample_shots_noalloc(gmps_batch* b, const int64_t* shots, int32_t shots_len, uint64_t seed,
                         uint64_t* out_bits, int64_t* out_hits);

/* Eq. (5): amplitudes <x|psi_inst> / ||psi_inst|| of the normalised state for cnt basis
 * indices (the stored chain's norm differs from 1 by the rounding of its tensors). xs: host
 * [cnt]; out_reim: host [2*cnt] (re, im). Queries pass through the workspace's staging region in
 * chunks. Synchronises. GMPS_E_NUMERIC if the norm is not finite and positive. */
int gmps_amplitudes(gmps_batch* b, int32_t inst, const uint64_t* xs, int64_t cnt,
                    double* out_reim);

/* <s|psi_inst> / ||psi_inst|| with |s> = |+>^n the uniform superposition (Eq. (2)). With the
 * marked amplitudes it fixes the state's components along the two directions of Eq. (5), the
 * normalised uniform superpositions over the marked and the unmarked indices, and so its
 * rotation angle. out_reim: host [2]. Synchronises. */
int gmps_overlap_uniform(gmps_batch* b, int32_t inst, double* out_reim);

/* The launch plan grover_iterate uses, as chosen by gmps_autotune. */
typedef struct {
  int32_t pipeline;     /* 1: pipelined sweeps, -1: sequential sweeps                      */
  int32_t precontract;  /* 1: pre-contracted reflections, -1: one bond-2 MPO per projector */
  int32_t waves_per_cu; /* workgroups per CU and class kernel; 0: the occupancy limit      */
  int32_t cached;       /* 1: taken from the cache file, 0: timed in this call             */
  int32_t candidates;   /* plans this batch allows                                         */
  int32_t reserved;
  double ms;            /* probe time of the plan (timed in this call or when cached)      */
} gmps_plan;

/* Batch orchestration: picks grover_iterate's launch plan by timing short runs of every plan
 * that keeps this batch's parity -- pipelined and sequential sweeps (pipelined only where
 * gmps_options.pipeline may apply), pre-contracted reflections (GMPS_FP64 and lossless bond
 * caps up to 17 only; on GMPS_MIXED their rotation angle drifts), and 0, 1 or 2 workgroups per CU and class
 * kernel -- and switches the batch to the fastest. k: host, k_len == 1 or B, the iteration
 * counts of the run to be tuned for; each probe scales them so that the longest chain runs
 * probe_iters (>= 1) iterations; a plan's time is the minimum of three runs timed by HIP
 * events, after an untimed run that captures its graph. cache_path (may be NULL): a text file of "key pipeline precontract waves_per_cu ms"
 * lines; the key hashes the device, the library's device sources, the precision, the kernel
 * and the batch's (class, n, M, probe k) multiset. A cached plan is applied without timing; a
 * timed one is appended (file errors are ignored). Leaves every instance at |s>, as
 * mps_init_uniform does. out (may be NULL): the plan. Synchronises. Errors: GMPS_E_ARG,
 * GMPS_E_HIP. */
int gmps_autotune(gmps_batch* b, const int64_t* k, int32_t k_len, int32_t probe_iters, const char* cache_path,
                  gmps_plan* out);

/* Checkpoint and resume: the whole state of a batch (every chain as stored, its bonds, edge
 * slots and warm-start records, and each instance's iteration count and diagnostics) copied to
 * or from host memory the caller owns, so that a long run can stop and continue in another
 * process (the warm-start records are held only when the batch's kernels read them).
 * gmps_state_bytes: the size of a checkpoint of this batch (0 for NULL). export: host
 * buffer of at least that many bytes; synchronises. import: a checkpoint exported from a batch
 * created with the same instances, precision and kernel (anything else is refused with
 * GMPS_E_ARG before any device memory is written); synchronises. Errors: GMPS_E_ARG,
 * GMPS_E_HIP. */
size_t gmps_state_bytes(const gmps_batch* b);
int gmps_state_export(gmps_batch* b, void* host, size_t bytes);
int gmps_state_import(gmps_batch* b, const void* host, size_t bytes);

/* Per-instance diagnostics; any pointer may be NULL. Synchronises.
 *  norm_drift:   host [B], largest |norm - 1| seen before a renormalisation
 *  trunc_weight: host [B], largest fraction of weight dropped by one truncation
 *  bond_dims:    host [B*64], bond_dims[i*64 + l] = bond l of instance i (l = 0..n)
 *  status:       host [B], GMPS_ST_* bits
 *  k_done:       host [B], iterations applied since mps_init_uniform
 *  flops:        host [2*B], algorithmic FP64 and FP32 flops spent by grover_iterate
 *                since mps_init_uniform (LAPACK-style counts at the actual tile sizes) */
int gmps_diagnostics(gmps_batch* b, double* norm_drift, double* trunc_weight, int32_t* bond_dims,
                     int32_t* status, int64_t* k_done, double* flops);

/* Milliseconds taken by the last grover_iterate() launch on the batch's stream, measured
 * with HIP events recorded around that launch. Synchronises. */
int gmps_last_iterate_ms(gmps_batch* b, double* ms);

/* Frees the handle (not the workspace). NULL is OK. */
int gmps_destroy(gmps_batch* b);

/* Static string for a GMPS_* status code. */
const char* gmps_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* GMPS_H */

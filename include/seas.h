/*
 * seas.h -- C ABI of the MI355X stress-transfer library for 2-D antiplane
 * fault networks (Ciardo & Romanet, "A divide-and-conquer strategy for fast
 * elastodynamic simulation of earthquakes and aseismic slip on fault networks").
 *
 * The library evaluates, every time step, the history functional f of the
 * elastic traction (the part of tau_el that is not radiation damping, Section
 * 2.3, eq. "superimposition2") on every element of a network of straight
 * faults, as the sum of
 *   - a non-replicating spectral self term per fault (Section 2.3.1, eqs.
 *     "functional_no_replication", "non_replicant_kernel",
 *     "funcational_discretized_form", "mode_dependent_truncation"), and
 *   - a fault-to-fault space-time convolution over a selective H-matrix, one
 *     binary cluster tree per fault, low-rank admissible blocks, dense
 *     near-field blocks, causality-truncated lag windows (Section 2.3.2, eqs.
 *     "fault-to-fault_interactions_discretized", "kernel_interactions",
 *     "primitives", "early_time", "admissibility_condition"),
 * and advances rate-and-state friction with the predictor-corrector of
 * Section 2.4 (eqs. "R&S_friction", "state_evolution_law", "force_balance").
 *
 * Conventions
 *   - Status codes: every call returns SEAS_OK (0) or a negative code; the
 *     message of the last failure on the calling thread is seas_last_error().
 *     No C++ exception crosses this boundary.
 *   - Units are SI. Element arrays are in fault order, element j of fault k at
 *     global index off_k + j (off_k = sum of earlier faults' n_elem).
 *   - Host pointers are read during the call only (copied). Device pointers
 *     (named *_dev) must stay valid until the work queued on `stream` is done.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Every call that takes a stream only enqueues work on it, except where
 *     stated; the library synchronises nothing else.
 *   - Objects: an operator is immutable after build and may be shared by
 *     several states; a state must be used from one stream at a time.
 *     The library owns the device memory of operators and states.
 */
#ifndef SEAS_H
#define SEAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t seas_status;
#define SEAS_OK 0
#define SEAS_ERR_INVALID_ARG (-1)   /* bad size, pointer, geometry or parameter */
#define SEAS_ERR_OOM (-2)           /* device or host allocation failed */
#define SEAS_ERR_HIP (-3)           /* a HIP runtime call failed */
#define SEAS_ERR_NOT_CONVERGED (-4) /* Newton did not converge (see seas_state_check) */
#define SEAS_ERR_MISMATCH (-5)      /* object used in the wrong mode or with another operator */
#define SEAS_ERR_INTERNAL (-6)

/* Storage/compute precision of the interaction factors. F64: factors, history
 * operand and accumulation in FP64. F32: factors and history operand in FP32,
 * FP32 accumulation within a work item, FP64 across items. BF16 / F16: the lags
 * applied once per time block (and, for ensembles, every lag and the static
 * tail) of admissible blocks (with one variant) or of every block (ensembles)
 * are stored in 16 bits with one power-of-two FP32 scale per work item,
 * multiplied on the matrix cores against a 16-bit copy of the history with FP32
 * accumulation; F16 also scales each staged history panel (per variant in
 * ensembles) and projected panel by a power of two so that their values stay in
 * range. With one variant the lags applied every step and the far lags of
 * near-field blocks are kept in FP32; ensembles keep the same entries
 * (near-field blocks, lags below 16, the static tail) in FP32. BF16 ensembles
 * keep a BF16 copy of the rate history for their 16-bit products (their FP32
 * entries read the FP64 history); F16 ensembles an FP32 copy. State, self term,
 * friction and time integration are FP64 in every mode. */
#define SEAS_F64 0
#define SEAS_F32 1
#define SEAS_BF16 2
#define SEAS_F16 3

const char* seas_last_error(void);
const char* seas_version(void);
/* x rounded to the storage format of factor_dtype (round to nearest even) and
 * back: the host conversion the build applies to stored factor values. */
double seas_round_factor(double x, int32_t factor_dtype);

/* One straight fault: centroid (cx, cy), unit normal (nx, ny) = e2' of its
 * local frame, tangent e1' = e3 x e2' = (-ny, nx) (Section 3.1), length and
 * number of equal piecewise-constant elements (collocated at midpoints,
 * Section 2.3.1). */
typedef struct {
  double cx, cy, nx, ny, length;
  int32_t n_elem;
  int32_t reserved;
} seas_fault_t;

typedef struct {
  double mu;        /* shear modulus [Pa] */
  double cs;        /* shear-wave speed [m/s] */
  double beta;      /* dt = beta * min(dx) / cs, beta <= 1/2 (Section 2.3.1) */
  double eta_H;     /* admissibility factor (eq. "admissibility_condition") */
  double aca_tol;   /* relative Frobenius tolerance of the low-rank factors */
  double eta_tmin;  /* causality window safety factors (Section 2.3.2) */
  double eta_tmax;
  double eta_w;     /* lowest-mode self window factor, T_end(1) = eta_w L / cs */
  int32_t leaf;     /* eta_leaf: maximum elements in a leaf cluster */
  int32_t compress; /* 0: every block stored dense (uncompressed operator) */
  int32_t int_tail; /* 1: static stress of slip older than the pair window is kept; 0: dropped */
  int32_t q_w;      /* window modulation integer, 0 = round(N_p / 5) per fault */
  int32_t mode_cap; /* 0 = all N_p modes of the 2 N_p padded transform; else keep n <= mode_cap */
  int32_t factor_dtype; /* SEAS_F64, SEAS_F32, SEAS_BF16 or SEAS_F16 */
  int32_t n_threads;    /* host threads for the build (0 = all) */
  int32_t host_only;    /* 1: build on the host only (no device memory; for inspecting the
                           partition, windows, tables and factors); evaluation and state calls
                           then fail with MISMATCH */
  int32_t time_block;   /* S in {0 (= 1), 1, 2, 4, 8, 16, 32}: lags T >= S are applied once per S
                           steps to S history windows (a lag-T factor only needs rates at least
                           T steps old), lags 1..S-1 and the static tail every step; the sum is
                           the same, only its evaluation order changes. BF16 / F16 operators
                           with one variant need 16; with several variants, 0 or 1; 32 needs
                           F32 factors (the 32-column matrix-core products) */
  int32_t n_variants;   /* 0 or 1: one friction parameter set; 16, 32 or 64: an ensemble of that
                           many parameter sets on this geometry (BF16 / F16 only), whose
                           interaction sums are one product of the factors with the
                           variants' histories side by side */
  int32_t state_update; /* states of this operator: 0 = the explicit update of Section 2.4 as
                           printed (theta* = theta + dt thetadot; the corrector with the averaged
                           state rate); 1 = the state law of eq. "state_evolution_law" integrated
                           in closed form over the step at constant slip rate (V in the
                           predictor, the averaged rate in the corrector), which keeps theta > 0
                           when the rate jumps by decades in one step (the explicit form cannot
                           start the two-fault benchmark of Section 3.1) */
  int32_t cluster_windows; /* 0: the causality window of Section 2.3.2 per fault pair; 1: per
                           H-matrix block (the cluster-level truncation Section 4.3 proposes):
                           a block's upper lag follows the pair rule applied to its clusters
                           (source midpoints to the receiver cluster's end points), at most the
                           pair's, and slip older than it contributes the block's static stress
                           (with int_tail); seas_operator_blocks reports each block's upper lag */
  int32_t adaptive_dt;  /* 0: every step is Delta t_min; 1: step 1 of Section 2.4.1: each step is
                           gamma Delta t_min with gamma = ceil(min_i adapt_xi Dc_i / V_i / Delta t_min)
                           (at least 1, at most gamma_max; the minimum over all variants), the rate
                           and slip histories kept on the Delta t_min grid (needs time_block 0/1) */
  int32_t gamma_max;    /* largest gamma (0 = 2^20) */
  double adapt_xi;      /* xi of the rule (0 = 0.5); the paper ties it to each element's stiffness
                           and friction through a formula it does not print, so it is an input here */
  int32_t free_surface; /* 1: a traction-free surface on the line y = surface_y, the medium below it
                           (y < surface_y), by the method of images (exact in anti-plane, the
                           construction of Appendix A's BP1-FD check): every source fault acts
                           also through its mirror image, with the slip continued across the
                           surface; each receiver fault therefore also has a pair with its own
                           image. Faults must lie below the line (end points may touch it). */
  int32_t reserved_fs;
  double surface_y;
  int32_t self_tail;    /* 0: the self term of eq. "funcational_discretized_form" as printed, each
                           mode's kernel cut after the cell of lag W_n; 1: slip older than the
                           window responds with the rest of the kernel, R_n D_n^{t-W_n-1},
                           R_n = |k_n| int over t >= (W_n + 1/2) dt of K(n, t) (the static tail
                           the cut drops; with it a slip held longer than the windows gives the
                           fault's static stress). Not in the paper: an optional correction */
  int32_t aca_partial;  /* 0: every admissible block-lag is evaluated whole and compressed by ACA
                           with full pivoting; 1: the lags at which every entry of an admissible
                           block lies behind both wave fronts (cs T dt beyond the largest distance
                           from a receiver midpoint to a source element edge) are compressed by
                           ACA with partial pivoting to aca_tol / 4, from rows and columns of
                           the block evaluated on demand (the cheaper construction the paper's
                           outlook proposes in place of its SVD; the convergence estimate is
                           checked on rows and columns spread over the block), then the SVD of
                           the crosses truncated at 3 aca_tol / 4. Earlier lags, near-field
                           blocks and static tails are built as with 0 (bit for bit) */
} seas_params_t;

typedef struct seas_op seas_op_t;
typedef struct seas_state seas_state_t;

/* Build the operator and upload it to the current HIP device: fault geometry
 * and the time step dt = beta min(dx) / cs (Section 2.3.1, Section 3.1), the
 * causality window [T_init, T_end] of every ordered fault pair (Section 2.3.2,
 * eq. "early_time" and the truncation paragraph), the kernel entries of eq.
 * "kernel_interactions" from the closed-form primitives of eq. "primitives",
 * the selective H-matrix of each pair (one binary cluster tree per fault,
 * bounding circles, eq. "admissibility_condition", dual-tree traversal),
 * low-rank compression of admissible blocks lag by lag (ACA in place of the
 * paper's truncated SVD, which Section 4.3 lists as an improvement), and the
 * self-kernel tables K_n^T with the mode windows W_n of eqs.
 * "non_replicant_kernel", "funcational_discretized_form" and
 * "mode_dependent_truncation". Blocking. The operator is owned by the caller
 * until seas_operator_destroy. Errors: INVALID_ARG for degenerate faults (length <= 0, n_elem < 2,
 * zero normal, a collocation point on another fault's element edge), OOM, HIP.
 * F32 operators with time_block 16 store the lags >= 16 for the matrix-core
 * segment kernel (rows grouped per workgroup); two environment variables, read
 * here, select other kernels for diagnosis: SEAS_NO_SEG=1 the one-item-per-
 * workgroup matrix-core kernel, SEAS_NO_MFMA=1 the vector-ALU kernel. The sums
 * agree to FP32 rounding. */
seas_status seas_build_operator(const seas_fault_t* faults, int32_t n_faults,
                                const seas_params_t* params, seas_op_t** out);
void seas_operator_destroy(seas_op_t* op);

typedef struct {
  int32_t n_faults, n_elem;   /* faults, total elements N */
  double dt;                  /* time step [s] */
  int32_t max_lag;            /* largest interaction lag T_end over pairs */
  int32_t max_self_window;    /* largest self window W_n over faults and modes (W_n + 1 with
                                 self_tail: the oldest lag the self term reads) */
  int64_t n_blocks;           /* H-matrix blocks over all ordered pairs */
  int64_t n_items;            /* work items applied once per time block */
  int64_t dense_entries;      /* entries of the uncompressed kernel in the pair windows */
  int64_t stored_entries;     /* stored factor entries (low rank + dense), lags >= 1 and tail */
  int64_t lag0_nnz;           /* nonzeros of the lag-0 interaction (pairs with T_init = 0) */
  int64_t self_entries;       /* sum over faults and modes of (W_n + 1), + 1 each with self_tail */
  double bytes_per_step;      /* algorithmic HBM bytes of one stress evaluation */
  double flops_per_step;      /* 2 x stored entries + self term MACs */
  double build_seconds;
  int32_t factor_dtype;
  int32_t time_block;         /* S of the build */
  int64_t far_entries;        /* stored entries applied once per time block (lags >= S) */
  int64_t n_items_near;       /* work items applied every step (lags 1..S-1, static tail) */
  int32_t n_variants;         /* variants a state of this operator holds */
  int32_t ncols;              /* columns of the far-list products: time_block x n_variants */
  int64_t n_segments;         /* BF16 / F16: workgroups of the far list (items with the same rows) */
  int64_t far_bytes;          /* bytes of the stored far-list factors (with the 16-bit row padding) */
  int64_t far_entries_f32;    /* BF16 / F16 with one variant: far entries of near-field (not
                                 admissible) blocks, kept in FP32 (included in far_entries);
                                 ensembles: the entries of their FP32 list */
  int64_t partial_bytes;      /* device bytes of the partial sums one interaction evaluation
                                 writes (see seas_eval_prescribed_noalloc) */
  int64_t far_entries_first;  /* time_block S > 1: far entries of lags S..2S-1 (the block-start
                                 items; included in far_entries) */
  int64_t far_entries_first_f32; /* the part of far_entries_first kept in FP32 by 16-bit builds */
} seas_op_info_t;

seas_status seas_operator_info(const seas_op_t* op, seas_op_info_t* out);

/* Causality window [T_init, T_end] (in lags) of every ordered pair (a, b),
 * a != b, row-major over a then b with the diagonal skipped:
 * n_faults * (n_faults - 1) entries each. */
seas_status seas_operator_windows(const seas_op_t* op, int32_t* T_init, int32_t* T_end);
/* Causality window [T_init, T_end] of one pair: b < n_faults the fault pair (a, b),
 * b in [n_faults, 2 n_faults) the pair of receiver fault a with the mirror image of
 * fault b - n_faults (free_surface; seas_operator_windows lists the fault pairs
 * only). The same index also selects image pairs in seas_operator_blocks.
 * INVALID_ARG for a pair that does not exist. */
seas_status seas_operator_pair_window(const seas_op_t* op, int32_t a, int32_t b, int32_t* T_init, int32_t* T_end);

/* Block partition of the ordered pair (a, b) (the dual-tree traversal of
 * Section 2.3.2): count (blocks == NULL) or copy rows of 6 int32: r0, r1, s0, s1
 * (element ranges local to the faults), 1 for admissible / 0 for near-field, and
 * the block's upper lag (the pair's T_end, or its own with cluster_windows), in
 * depth-first traversal order. */
seas_status seas_operator_blocks(const seas_op_t* op, int32_t a, int32_t b,
                                 int32_t* blocks, int64_t* count);

/* Self-kernel table K_n^T of fault k, mode n (1..), T = 0..W_n, and W_n.
 * Host copy of the values the device uses. With self_tail = 1 the table has one
 * more entry, out[W_n + 1] = R_n (the tail coefficient applied to D_n^{t-W_n-1});
 * capacity must then be at least W_n + 2. */
seas_status seas_operator_self_table(const seas_op_t* op, int32_t k, int32_t n,
                                     double* out, int32_t capacity, int32_t* W_n);

/* Reconstruct the kernel matrix of the ordered pair (a, b) at lag T (T >= 0; T = -1
 * for the static-tail matrix, stored as -G/eta with G the static stress per unit
 * slip) from the stored factors: out is n_elem(a) x n_elem(b), row-major, host.
 * b = n_faults + a selects the pair of fault a with its own mirror image
 * (free_surface; the image pair's sign included). With free_surface, the pair
 * (a, b) for b < n_faults is what the evaluation applies to the slip of b: the
 * kernel against fault b plus the one against its image (sign included), each
 * inside its own window. Only for operators built with host_only = 1 (the factors
 * are on the host). */
seas_status seas_operator_lag_matrix(const seas_op_t* op, int32_t a, int32_t b, int32_t T, double* out);

/* Rate-and-state parameters, one value per element and variant (host arrays of
 * n_variants x N, variant-major):
 * strength sigma_n [f0 + a ln(V/V0) + b ln(V0 theta / Dc)], state law with
 * exponent eps (1 = aging law). */
typedef struct {
  const double *a, *b, *Dc, *sigma_n, *V0, *f0, *eps;  /* eps may be NULL (aging law) */
} seas_friction_t;

/* Device bytes a state of `n_variants` variants needs (admission control). */
size_t seas_state_bytes(const seas_op_t* op, int32_t n_variants);

/* Create a state at t = 0 (the unknowns of Section 2.4: slip, slip rate,
 * state variable, with the background stress tau0 of eq. "force_balance"):
 * slip rate V_init, state theta_init, background shear stress tau0 and its
 * rate (may be NULL; tectonic loading as in Section 3.2), slip delta_init (may
 * be NULL = 0). Host arrays of n_variants x N (variant-major). Histories before t = 0
 * are zero (no prior slip) unless seas_state_load_history is called next.
 * n_variants must equal the operator's (seas_op_info_t.n_variants); every
 * variant evolves on its own, and the variants share the operator's factors. */
seas_status seas_state_create(seas_op_t* op, int32_t n_variants, const seas_friction_t* fric,
                              const double* V_init, const double* theta_init,
                              const double* tau0, const double* tau0_rate,
                              const double* delta_init, void* stream, seas_state_t** out);
/* Free the state's device memory and its second stream (after waiting for that
 * stream). Work still queued on the caller's streams that uses the state must
 * have finished: synchronise them first. NULL is ignored. */
void seas_state_destroy(seas_state_t* st);

/* Prior slip-rate history V[m][n_variants][N] for the n_hist steps before t = 0
 * (host, oldest first): fills both histories (slip before t = 0 follows from
 * delta^{m+1} = delta^m + dt V^m) and the expired-slip accumulators. Must be
 * called right after seas_state_create. */
seas_status seas_state_load_history(seas_state_t* st, const double* V_hist, int32_t n_hist,
                                    void* stream);

/* Start a new window in one variant slot of a stepping (or fresh) state: the
 * slot's friction parameters, slip rate, state, background stress and its rate
 * and slip (host arrays of N; tau0_rate, delta_init and fric->eps may be NULL)
 * replace the old ones, its rate and coefficient histories and expired-slip
 * accumulators are cleared, and the slot's time origin becomes the current step
 * (its loading rate counts from there). The other variants are untouched and
 * keep stepping; the slot evolves exactly as a fresh state would from t = 0.
 * For continuous batching of requests that share a geometry. Synchronises the
 * stream. */
seas_status seas_state_reset_variant(seas_state_t* st, int32_t variant, const seas_friction_t* fric,
                                     const double* V_init, const double* theta_init, const double* tau0,
                                     const double* tau0_rate, const double* delta_init, void* stream);
/* Stress evaluation of a prescribed slip-rate history (no friction): the
 * history functional f of eq. "superimposition2", split as in eq.
 * "traction_decomposition" into the spectral self term of each fault (eq.
 * "funcational_discretized_form") and the fault-to-fault sum of eq.
 * "fault-to-fault_interactions_discretized". For
 * n = 1..n_steps, with V^m = V_dev[m][variant][element] (device, FP64,
 * n_steps x n_variants x N):
 *   delta^n = delta^{n-1} + dt V^{n-1}
 *   f^n = f_self(D^n, D^{n-1}, ...) + f_int(V^{n-1}, V^{n-2}, ...)
 * written to f_dev[n-1][variant][element] (device, FP64). Consecutive calls continue the
 * same history. MISMATCH if the state has taken SEAS steps. */
seas_status seas_eval_prescribed(seas_op_t* op, seas_state_t* st, const double* V_dev,
                                 int32_t n_steps, double* f_dev, void* stream);

/* seas_eval_prescribed for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, bit for bit, but the partial sums
 * of the interaction evaluation live in a fixed 32 MiB device array of the
 * library (one per GPU, held until the process ends) instead of the state's
 * buffers, and the call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine; the state and operator were allocated at set-up). The
 * caller passes inputs and outputs as for seas_eval_prescribed. Every partial
 * sum is written before it is read, so nothing is cleared between calls; the
 * array keeps the last call's contents. Calls that overlap on one GPU (any
 * states, any streams) share the array and race: order them. Errors:
 * INVALID_ARG when the operator's partial sums (seas_op_info_t.partial_bytes)
 * exceed 32 MiB, MISMATCH when kernel timing is on for the state (timing
 * creates events), and those of seas_eval_prescribed. */
seas_status seas_eval_prescribed_noalloc(seas_op_t* op, seas_state_t* st, const double* V_dev, int32_t n_steps,
                                         double* f_dev, void* stream);

/* Advance n_steps predictor-corrector steps (Section 2.4, steps 2 and 3: the
 * predictor, the Newton solve of the force balance with the friction of eq.
 * "R&S_friction", the state law of eq. "state_evolution_law", the corrector
 * with averaged rates, and the history append). Enqueue only.
 * Newton failure (a solve that needs more than 50 iterations, or meets a
 * non-finite force balance, e.g. a non-finite background stress): the variant's
 * commits stop at the failing step, so its slip, rate, state, histories and
 * expired-slip accumulators stay at its last good step, and the rest of the
 * enqueued steps leave it untouched; the other variants keep stepping. The
 * failure is reported by seas_state_check / seas_state_variant_status. Part of each step (the
 * self history and the predictor transform) runs on a second stream the state
 * creates on first use (default priority), forked from and joined back into
 * `stream` by events within the step: when the call returns, all of its work is
 * ordered on `stream` like the rest of the library's calls. */
seas_status seas_step(seas_op_t* op, seas_state_t* st, int32_t n_steps, void* stream);

/* Synchronise `stream` and report NOT_CONVERGED if a variant's Newton solve
 * failed (message: the variants and the steps they are held at). With one
 * variant the state is then at its last good step: the step index goes back to
 * it, the flag is cleared and stepping may resume from there (e.g. after
 * seas_write_state). With several variants the variants share one clock, so a
 * failed variant stays held (its histories fall behind the others') and keeps
 * being reported until seas_state_reset_variant starts a new window in its
 * slot. */
seas_status seas_state_check(seas_state_t* st, void* stream);
/* Per-variant convergence (synchronises `stream`): failed[v] = 1 if variant v
 * is held after a Newton failure, good_step[v] = the step index of its last
 * committed step (either pointer may be NULL; host arrays of n_variants). */
seas_status seas_state_variant_status(const seas_state_t* st, int32_t* failed, int64_t* good_step, void* stream);

#define SEAS_FIELD_V 0          /* slip rate at the current step */
#define SEAS_FIELD_THETA 1
#define SEAS_FIELD_DELTA 2      /* slip */
#define SEAS_FIELD_THETADOT 3
#define SEAS_FIELD_F_HIST 4     /* interaction history part (lags >= 1 + tail) of the last step */
#define SEAS_FIELD_F_SELF 5     /* self term of the last corrector */
#define SEAS_FIELD_F_INT 6      /* interaction stress of the last corrector (with lag 0) */
#define SEAS_FIELD_TAU0 7

/* Copy the N values of a field of one variant to dst (device if dst_is_device,
 * else host; a host copy synchronises the stream): the unknowns of the step of
 * Section 2.4 (slip, slip rate, state, state rate) and the parts of the
 * traction of eqs. "superimposition2" and "traction_decomposition".
 * count must equal N (INVALID_ARG otherwise). */
seas_status seas_read_state(const seas_state_t* st, int32_t field, int32_t variant, double* dst,
                            size_t count, int32_t dst_is_device, void* stream);
/* Overwrite a field of one variant at the current step, e.g. to resume from
 * values saved elsewhere or to continue after a Newton failure (Section 2.4
 * unknowns): SEAS_FIELD_V (> 0; also the newest row of the rate history, which
 * the next steps read at lag 1), SEAS_FIELD_THETA (> 0), SEAS_FIELD_DELTA (also
 * the newest row of slip coefficients of the self term) or SEAS_FIELD_TAU0;
 * writing V or THETA recomputes the state rate. src holds N values (device if
 * src_is_device, else host); count must equal N. Synchronises the stream.
 * Errors: INVALID_ARG (other fields, bad count or values), MISMATCH (a
 * prescribed-history state). */
seas_status seas_write_state(seas_state_t* st, int32_t field, int32_t variant, const double* src, size_t count,
                             int32_t src_is_device, void* stream);
/* Device time of the interaction-evaluation kernel: when enabled, every launch of
 * it inside seas_step / seas_eval_prescribed is bracketed by HIP events recorded
 * on the launch stream. With time_block S > 1 the timed launch is the far part
 * with lags >= 2S (seas_op_info_t.far_entries - far_entries_first entries), one
 * per time block; the block-start items (lags S..2S-1) are not timed. In the plain
 * form every far launch is timed. read_timing synchronises `stream`, returns the
 * summed milliseconds and the number of launches since the last read, and resets
 * them. */
seas_status seas_state_set_timing(seas_state_t* st, int32_t enable);

/* Block lookahead of seas_step (time_block S > 1; on by default). The stress at
 * the S steps of a time block from lags >= 2S needs rates up to the step before
 * the previous block only (Section 2.4 evaluates the history sum from stored
 * rates; eq. "fault-to-fault_interactions_discretized"), so seas_step launches
 * that part for the next block on a second stream of its own as soon as the
 * current block's far sums are reduced, and it runs beside the current block's
 * steps; the next block waits for it and adds its lags S..2S-1. A lookahead is
 * only started for a block the same seas_step call reaches, so every call leaves
 * no work behind on that stream. enable = 0 applies both parts at each block
 * start on the caller's stream. The sums are identical either way. The lookahead
 * stream is non-blocking, so a caller's stream of any kind overlaps with it. */
seas_status seas_state_set_overlap(seas_state_t* st, int32_t enable);

/* Tile tuning of the far pass on the operator's own factors. Operators on the
 * matrix-core segment kernel (FP32 with time_block 16 or 32, BF16 / FP16 with one
 * variant or ensembles) have 3 compiled variants of it, which differ in how far
 * ahead the global operand is loaded and, for FP32, in how many waves per SIMD their
 * registers are fitted to (FP32 0: 2 steps ahead, 4 waves; 1: 2 steps, 3 waves; 2: 3
 * steps, 3 waves; 16-bit 0: 8 steps; 1: 4; 2: 12); every variant computes the same
 * sums in the same order, so results are identical. seas_operator_tune times the
 * far launch of a whole time block (the lags >= 2S; ensembles: the whole far list of
 * a step, whose FP32 list is not tuned) of each variant on the state's current history,
 * reps launches each after one untimed, on the stream (it synchronises), writes the
 * average milliseconds per launch to ms[0..2] and selects the fastest (*choice) for
 * every later launch of the operator; the state's fields are not changed (only its
 * partial-sum buffer, which the next time block rewrites). Other operators have one
 * form: ms[] = -1 and *choice = the current variant. The choice is a setting of the
 * operator, read when a far launch is enqueued: tune or set it while no other thread
 * enqueues steps of the operator's states. A graph captured before keeps the variant
 * it recorded. ms and choice may be NULL. INVALID_ARG for reps < 1, MISMATCH for a
 * state of another operator. seas_operator_set_tune selects a variant directly
 * (INVALID_ARG outside 0..2). */
seas_status seas_operator_tune(seas_op_t* op, seas_state_t* st, void* stream, int32_t reps, double* ms,
                               int32_t* choice);
seas_status seas_operator_set_tune(seas_op_t* op, int32_t variant);

/* Captured steps: with enable = 1, seas_step runs the fixed steps that fill whole
 * time blocks (S steps; 16 steps when every step applies the far list, S = 1 or
 * seas_state_set_time_block(1)) as replays of one HIP graph per state, captured at
 * its first use on a stream of the state's own and launched on the caller's
 * stream; steps before the next block start and a remainder shorter than a block
 * run as before. Every step evaluates exactly as an uncaptured one: the captured
 * kernels read the step base from a device word of the state that the graph
 * itself advances, so one graph serves every block. The block lookahead and
 * kernel timing do not apply inside a replay. The graph holds the state's and
 * the operator's device pointers: it is recaptured when the evaluation order
 * changes and released with the state. Graph launches remove the per-kernel
 * launch cost of a step (about 14 kernels), which is what bounds small networks.
 * MISMATCH for states of an adaptive operator (each step's length is chosen on
 * the host); enable = 0 returns to plain launches. */
seas_status seas_state_set_graph(seas_state_t* st, int32_t enable);

/* Graph replays launched by seas_step since the state was created, and the steps
 * per replay of its current graph (0 before the first capture). Either output may
 * be NULL. */
seas_status seas_state_graph_info(const seas_state_t* st, int64_t* replays, int32_t* steps_per_replay);

/* Evaluation order of a state built with time_block S > 1: S (default) applies the
 * lags >= S once per S steps; 1 applies them every step (the plain per-step form).
 * Results agree to rounding; used to compare both forms on one operator. */
seas_status seas_state_set_time_block(seas_state_t* st, int32_t S);
seas_status seas_state_read_timing(seas_state_t* st, void* stream, double* ms_total, int64_t* launches);

/* Current step index: the grid time t / Delta t_min reached (with fixed steps the
 * number of steps taken, or of prescribed steps evaluated). */
int64_t seas_state_step_index(const seas_state_t* st);

/* Progress of a stepping state (adaptive steps, seas_params_t.adaptive_dt): steps
 * taken by seas_step, gamma of the last one, and the time reached in seconds
 * (grid index times Delta t_min). Any output may be NULL. */
seas_status seas_state_progress(const seas_state_t* st, int64_t* steps_taken, int64_t* last_gamma, double* time_s);

/* Adaptive steps: a cap on gamma for this state below the operator's gamma_max (0
 * removes it). The rule reads the rates of the current state, which must balance
 * the stresses: from an initial state that does not (a rate held while an
 * overstress is applied, as in Section 3.1), the first steps are taken with cap 1
 * and the cap is lifted once the solves have set the rates. INVALID_ARG for
 * cap < 0. */
seas_status seas_state_set_gamma_cap(seas_state_t* st, int64_t cap);

/* Checkpoint: size in bytes, save to / restore from a host buffer (synchronises
 * the stream). Restoring into a state of the same operator reproduces the
 * saved state exactly. */
size_t seas_state_checkpoint_bytes(const seas_state_t* st);
seas_status seas_state_save(const seas_state_t* st, void* host_buf, size_t bytes, void* stream);
seas_status seas_state_restore(seas_state_t* st, const void* host_buf, size_t bytes, void* stream);

/* ---------------------------------------------------------------- serving
 * A request loop for simulation windows on several geometries ("pools", one
 * operator each, built with n_variants slots). Each pool steps one ensemble
 * state on its own stream, in chunks of at most chunk_steps steps; requests of
 * a pool join free variant slots between chunks (seas_state_reset_variant) and
 * leave when their window ends, so a running batch admits new requests while
 * others are on the GPU. A pool's state is created when its first request
 * arrives and the sum of the states' bytes (seas_state_bytes) stays within
 * device_budget; an idle pool gives its memory back when another pool waits
 * for it. Requests queue per pool in arrival order. A slot whose Newton solve
 * fails ends its request with NOT_CONVERGED and the outputs of its last good
 * step; the other slots are not affected. Not an accuracy feature:
 * a request's result is the one it gets alone in a fresh state, bit for bit
 * (every slot's product column is formed on its own, FP16 history panels with
 * a power-of-two scale per slot). */
typedef struct {
  int32_t pool;           /* index of the request's operator in seas_server_create */
  int32_t n_steps;        /* window length in steps (>= 1) */
  double arrival_s;       /* arrival time in seconds after seas_server_run starts */
  seas_friction_t fric;   /* N values each (host, read during the run) */
  const double *V_init, *theta_init, *tau0;  /* N values (host) */
  const double *tau0_rate, *delta_init;      /* N values (host) or NULL */
  double *V_out, *theta_out, *delta_out;     /* N values (host) written when the window ends, or NULL */
  double admit_s;         /* out: time it took a slot */
  double finish_s;        /* out: time its results were copied out */
  int32_t status;         /* out: SEAS_OK, or the error its pool reported (e.g. NOT_CONVERGED) */
  int32_t reserved;
} seas_request_t;
typedef struct seas_server seas_server_t;
/* ops: n_ops operators (not owned; must outlive the server); idle: one request
 * per pool whose friction and initial values fill the slots no request holds
 * (a quiet, steady window, so that idle slots neither diverge nor fail). */
seas_status seas_server_create(seas_op_t* const* ops, int32_t n_ops, const seas_request_t* idle,
                               size_t device_budget, int32_t chunk_steps, seas_server_t** out);
/* Play a trace of n_reqs requests in real time and return when all are done.
 * Blocking; fills admit_s, finish_s and status of every request. A request
 * whose slot fails a Newton solve ends with NOT_CONVERGED when the chunk that
 * failed completes; its outputs hold its last good step and its slot returns
 * to the idle window. Errors of the call itself: INVALID_ARG (a
 * request with a bad pool index or n_steps < 1), HIP, INTERNAL (requests left
 * that no pool can admit). */
seas_status seas_server_run(seas_server_t* sv, seas_request_t* reqs, int32_t n_reqs);
void seas_server_destroy(seas_server_t* sv);

#ifdef __cplusplus
}
#endif
#endif /* SEAS_H */

/*
 * frg.h -- C ABI of libfrg, the MI355X (gfx950) engine for the right-hand side
 * of the discretised one-loop fRG flow of the 2D Hubbard four-point vertex.
 *
 * The paper (Rohe, "Hierarchical Parallelisation of Functional Renormalisation
 * Group Calculations - hp-fRG") states the problem in Sec. 2, Eq. (1):
 * all discretised couplings live in one flat array V[i] that obeys
 * dV[i]/dg = F[V[j]; g], integrated by an explicit stepper so that F is
 * computed for every component with V frozen, after which the step is taken.
 * Sec. 4 fixes the instance: the square-lattice Hubbard model (hoppings t, t',
 * chemical potential mu), three one-loop diagrams (particle-particle, direct
 * and crossed particle-hole) integrated over the Brillouin zone, N patches.
 * Here the flow parameter is the temperature: F = dV/dT, integrated in
 * s = ln T.
 *
 * Conventions shared by every call:
 *  - Every call returns frg_status; no C++ exception crosses the ABI.
 *    Argument errors are detected on the host before anything is enqueued and
 *    leave device memory untouched.  Device errors surface as FRG_EDEVICE at
 *    the call that detects them (launch errors at once, faults at the next
 *    synchronising call).  frg_last_error() gives a thread-local message.
 *  - Pointers named d_* are device pointers owned by the caller, 256-byte
 *    aligned (any hipMalloc / torch CUDA allocation is), sized by frg_sizes.
 *    The context owns its geometry tables and workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work is enqueued asynchronously on it; frg_flow synchronises once
 *    per step to read one status word.
 *  - V and F are [N][N][N] row-major FP64, V[j1][j2][j3] = V(k1,k2,k3) with
 *    k4 = k1 + k2 - k3.  F is dV/dT (not dV/ds).
 *  - Bubble tensors are [row][a][b] (a: patch of the fine-grid loop line,
 *    b: patch of the second line).  pp rows: pairs (i <= j) in lexicographic
 *    order, transfer q = k_i + k_j.  ph rows: row 0 is Q = 0; then pairs
 *    (x, y), x != y, lexicographic, transfer Q = k_x - k_y.
 *  - A context is not thread-safe; use one per stream.
 */
#ifndef FRG_H
#define FRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FRG_OK = 0,
    FRG_EINVAL = 1,      /* bad argument (detected before any launch) */
    FRG_ENOMEM = 2,      /* device or host allocation failed */
    FRG_EDEVICE = 3,     /* HIP runtime / kernel error */
    FRG_ENOTSUP = 4,     /* valid but unsupported size or mode */
    FRG_ENONFINITE = 5   /* a flow produced NaN/Inf */
} frg_status;

typedef enum {
    FRG_PREC_FP64 = 0,        /* FP64 bubbles, FP64 MFMA contraction */
    FRG_PREC_SPLIT_BF16 = 1   /* FP32 compensated bubbles, split-BF16 (hi+lo) MFMA, FP32 accumulate */
} frg_precision;

typedef enum { FRG_RK4 = 0, FRG_DP54 = 1 } frg_stepper;

typedef enum {
    FRG_STOP_NONE = 0,
    FRG_STOP_TMIN = 1,       /* reached T_min */
    FRG_STOP_DIVERGED = 2,   /* max|V| > vmax after an accepted step: a result, not an error */
    FRG_STOP_MAXSTEPS = 3,
    FRG_STOP_NONFINITE = 4,
    FRG_STOP_HMIN = 5        /* step size underflow */
} frg_stop;

/* Model: eps(k) = -2t(cos kx + cos ky) - 4t'(cos kx cos ky) - mu.
 * N patches, 4 <= N <= 256, N % 4 == 0; n_rad x n_ang fine points per patch,
 * 1 <= n_rad*n_ang <= 1024.  U is the bare coupling (V = U initially). */
typedef struct {
    double t, tp, mu, U;
    int32_t N, n_rad, n_ang;
} frg_params;

/* Flow options.  stepper RK4: fixed_steps uniform steps in s = ln T from T0
 * to T_min.  DP54: Dormand-Prince 5(4), first step h0 (in s, sign ignored:
 * always towards T_min), err = max|y5-y4|/(atol + rtol max(|y|,|y5|)),
 * accept if err <= 1, h <- h clamp(0.9 err^-1/5, 0.2, 5), last step clipped
 * onto T_min.  Both stop after an accepted step with max|V| > vmax.
 * max_steps > 0 caps accepted steps. */
typedef struct {
    frg_stepper stepper;
    frg_precision prec;
    double T0, T_min, rtol, atol, vmax, h0;
    int32_t fixed_steps, max_steps;
} frg_flow_opts;

typedef struct {
    frg_stop reason;
    double T_end;        /* temperature of the final state */
    double T_c;          /* T at the first accepted step with max|V| > vmax (NaN if none) */
    double T_c_interp;   /* crossing interpolated linearly in s */
    int32_t accepted, rejected, rhs_evals, first_step_rhs;
} frg_flow_result;

/* Device-side flow state used by frg_flow_step (FRG_STATE_LEN doubles). */
#define FRG_STATE_LEN 32
enum {
    FRG_ST_S = 0,          /* current s = ln T (g in an interaction flow) */
    FRG_ST_H = 1,          /* next step size */
    FRG_ST_ERR = 2,        /* error norm of the last attempt */
    FRG_ST_REASON = 3,     /* frg_stop of the flow (0 while running) */
    FRG_ST_ACCEPTED = 4,
    FRG_ST_REJECTED = 5,
    FRG_ST_RHS = 6,        /* rhs evaluations so far */
    FRG_ST_VMAX = 7,       /* max|V| of the current state */
    FRG_ST_SC = 8,         /* s at divergence */
    FRG_ST_SC_INTERP = 9,
    FRG_ST_FIRST_RHS = 10, /* rhs evaluations spent up to the first accepted step */
    FRG_ST_SMIN = 11,      /* target s = ln T_min */
    FRG_ST_FSAL = 12       /* 1 when the stored first-stage derivative is valid */
};

typedef struct frg_ctx_s *frg_ctx;

/* Build the host geometry (patch centres, sector boundaries, fine grid,
 * transfer momenta; plain FP64 on the host, no FP contraction), upload it,
 * and tabulate on the device the patch of every second loop line (one byte
 * per (row, fine point); temperature independent).  Cost: one-off.
 * Errors: EINVAL for bad parameters or out==NULL, ENOTSUP for n_f > 1024,
 * ENOMEM, EDEVICE (no gfx950 device). */
frg_status frg_create(const frg_params *p, frg_ctx *out);
frg_status frg_destroy(frg_ctx ctx);

/* Element counts: V/F entries (N^3), pp and ph bubble entries (rows*N*N),
 * and the device workspace the context holds. Any pointer may be NULL. */
frg_status frg_sizes(frg_ctx ctx, size_t *n_v, size_t *n_bpp, size_t *n_bph,
                     size_t *workspace_bytes);

/* Copy the host geometry out (host pointers, any may be NULL):
 * kc[N][2], bnd[N+1][2], fine[N*n_f][4] = (px, py, w, xi), qpp[Tpp][2],
 * qph[Tph][2], idx4[N][N][N] = patch of k1 + k2 - k3. */
frg_status frg_tables(frg_ctx ctx, double *kc, double *bnd, double *fine, double *qpp,
                      double *qph, int32_t *idx4);

/* Host-only: build the geometry for p and copy it out as frg_tables does,
 * without a context or a device (any output may be NULL). */
frg_status frg_host_tables(const frg_params *p, double *kc, double *bnd, double *fine,
                           double *qpp, double *qph, int32_t *idx4);

/* The paper's quadrature as the fine grid (Sec. 4: an outer fixed midpoint
 * grid in energy, an inner locally adaptive midpoint rule along each energy).
 * n_E shells at the midpoints of [eps(0,0), eps(pi,pi)] (the band for
 * |t'| < t/2); along each shell, per patch sector and octant piece of it, the
 * angles whose ray from Gamma reaches the shell energy are integrated by a
 * trisection midpoint rule in the ray angle, a cell cut in thirds while its
 * one- and three-point values differ by more than rtol * I_E * h / 2pi (I_E a
 * coarse estimate of the shell's whole inner integral, h the cell width), to
 * at most 3^max_level points per piece and shell.  Point weights are
 * dE h r / (d eps / dr) / (2pi)^2, not normalised.  p->n_rad and p->n_ang are
 * ignored.  Every patch holds n_f points (frg_points): its live points first,
 * then zero-weight padding; n_f is a multiple of 512.  Needs |t'| < t/2,
 * n_E >= 1, 1 <= max_level <= 12, rtol > 0 (EINVAL); ENOTSUP when a patch
 * would hold more than 131072 points; otherwise as frg_create.  Single flows
 * only (batches take polar grids). */
typedef struct {
    int32_t n_E, max_level;
    double rtol;
} frg_egrid;
frg_status frg_create_egrid(const frg_params *p, const frg_egrid *e, frg_ctx *out);

/* Points per patch: n_f, the table stride of a patch, and counts[N], each
 * patch's live points (n_f for every patch of a polar grid).  Either may be NULL. */
frg_status frg_points(frg_ctx ctx, int32_t *n_f, int32_t *counts);

/* Host-only frg_host_tables for the energy-angle grid: n_f and counts as
 * frg_points; call with fine = NULL first to learn n_f (fine holds N * n_f
 * rows). */
frg_status frg_host_tables_egrid(const frg_params *p, const frg_egrid *e, int32_t *n_f, int32_t *counts,
                                 double *kc, double *bnd, double *fine, double *qpp, double *qph,
                                 int32_t *idx4);

/* Copy the device table of second-line patches (kind 0 = ph, 1 = pp) into
 * d_out[rows][N*n_f] (uint8), points in the fine-grid order of frg_tables
 * (the device keeps each patch's points in its own order). */
frg_status frg_bins(frg_ctx ctx, int32_t kind, uint8_t *d_out, void *stream);

/* Bubble derivatives at temperature T > 0 (Sec. 4: the three one-loop
 * diagrams share two kinds of bubble):
 *   Bpp_q(a,b) = sum_{p in a, pi(q-p) = b} w_p dL_pp/dT(xi_p, eps(q-p))
 *   Bph_Q(a,b) = sum_{p in a, pi(p+Q) = b} w_p dL_ph/dT(xi_p, eps(p+Q))
 * FP64: d_bpp/d_bph are double; SPLIT_BF16: float (compensated sums).
 * Either output may be NULL. */
frg_status frg_bubbles(frg_ctx ctx, double T, frg_precision prec, void *d_bpp, void *d_bph,
                       void *stream);

/* The bubble rows as the rhs sweeps them under the C4v row reduction (Sec. 4
 * reduces the work with the lattice symmetries): one pp row q per C4v orbit of
 * the transfers, evaluated together with the ph row of -q (the two second
 * lines share one energy).  frg_bubble_reps gives their number and (host
 * arrays of n_rep entries, nullable) their pp and ph row indices in the
 * numbering of frg_bubbles; frg_bubbles_reps writes those rows, pp row i to
 * d_bpp[i] and its paired ph row to d_bph[i], each [n_rep][N][N] in FP64 or
 * FP32 by prec (the caller's device buffers).  ENOTSUP when the grid has no
 * reduction (N % 8 != 0); EINVAL for bad T or a null or misaligned output. */
frg_status frg_bubble_reps(frg_ctx ctx, int32_t *n_rep, int32_t *pp_rows, int32_t *ph_rows);
frg_status frg_bubbles_reps(frg_ctx ctx, double T, frg_precision prec, void *d_bpp, void *d_bph,
                            void *stream);

/* One rhs evaluation F = dV/dT at temperature T for all N^3 entries (Eq. (1)
 * with V frozen; the three one-loop channels).  d_V and d_F are [N][N][N]
 * FP64 and must not overlap. */
frg_status frg_rhs(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec,
                   void *stream);

/* frg_rhs for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, result and settings (symmetry, zero-chunk skipping,
 * symmetric-vertex mode) as frg_rhs, with the same kernels; the per-call
 * workspace (point factors, bubble rows, operand layout, channel partials)
 * lives in the library's static device scratch of FRG_NOALLOC_SCRATCH_BYTES
 * bytes instead of the context.  The call allocates nothing and needs no
 * earlier frg_rhs.  Every call on one device shares that device's scratch:
 * calls that overlap on one device (other streams, other threads, other
 * contexts) race and must be ordered by the caller.  Nothing in the scratch
 * needs to start at zero (each piece is written in full before it is read).
 * Returns ENOTSUP, before any launch, when the workspace of this context and
 * precision exceeds the scratch (e.g. N = 96 fits in symmetric-vertex mode,
 * not with every column computed in FP64) or with the self-energy on; other
 * errors as frg_rhs. */
#define FRG_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
frg_status frg_rhs_noalloc(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec,
                           void *stream);

/* Self-energy flowing with the vertex (Sec. 2 names self-energies as the
 * extension of the four-point flow and gives no form; the one here is a
 * reading): a static value S_j per patch, stored after the vertex, so that with
 * the switch on every V and F of frg_rhs, frg_flow_init, frg_flow_step and
 * frg_flow holds N^3 + N doubles ([V, S]).  Every loop line carries its patch's
 * S (the fine point's patch and the second line's), and
 *   dS_j/dT = sum_a D_a [2 V(j,a,j) - V(a,j,j)],
 *   D_a = sum_{p in a} w_p d/dT n_F((xi_p + S_a)/T)  (at fixed S),
 * in FP64 in both precisions.
 *   enable = 1: a general S; every bubble row is computed, unpaired.
 *   enable = 2: the caller's S is C4v invariant (S(g j) = S(j)), which a flow
 *               from a C4v-invariant V and S keeps: the bubble rows are then
 *               still C4v images of each other and pp/ph pairs, and the C4v
 *               row reduction applies as without a self-energy; so does the
 *               symmetric-vertex mode (frg_set_vsym), whose reduced flow
 *               state then carries S after its reduced entries.
 *               frg_flow_init checks S (EINVAL beyond 1e-12 relative); a
 *               direct frg_rhs call takes it on trust.  ENOTSUP on a grid
 *               without exact C4v covariance (N % 8 != 0).
 *   enable = 0: off.  Other values: EINVAL.
 * Polar and energy-angle grids, single flows only (ENOTSUP in a batch).
 * enable = 1 is refused (EINVAL) while the symmetric-vertex mode is on, and
 * frg_set_vsym(1) while a general self-energy is on.  Switching changes the
 * length of the flowing array: start flows again (frg_flow_init) afterwards.
 * The interaction flow (frg_rhs_full, frg_iflow*) ignores it.  Initial S = 0 is
 * the caller's.  frg_self_energy reports the switch (0, 1 or 2). */
frg_status frg_set_self_energy(frg_ctx ctx, int32_t enable);
frg_status frg_self_energy(frg_ctx ctx, int32_t *active);

/* Initialise a device flow state (FRG_STATE_LEN doubles) for o: s = ln T0,
 * h = first step, counters zero.  d_V is the initial vertex (unchanged). */
frg_status frg_flow_init(frg_ctx ctx, const frg_flow_opts *o, const double *d_V,
                         double *d_state, void *stream);

/* One step attempt (RK4: one step; DP54: one attempt, accepted or rejected)
 * of the explicit stepper of Eq. (1) in s = ln T, entirely on the device:
 * the stages, the FP64 error norm, the step control and the stop test read
 * and write d_state; nothing is synchronised.  Does nothing once
 * d_state[FRG_ST_REASON] != 0. */
frg_status frg_flow_step(frg_ctx ctx, const frg_flow_opts *o, double *d_V, double *d_state,
                         void *stream);

/* Whole flow from V0 (in d_V, overwritten with the final state) until a stop
 * condition.  d_log (nullable, device) receives 8 doubles per accepted step:
 * s, h, err, max|V|, rhs_evals, rejected, accepted, reason (up to
 * log_cap rows).  Synchronises once per step.  Returns FRG_ENONFINITE if the
 * state became non-finite (r->reason = FRG_STOP_NONFINITE). */
frg_status frg_flow(frg_ctx ctx, const frg_flow_opts *o, double *d_V, double *d_log,
                    int32_t log_cap, frg_flow_result *r, void *stream);

/* ---- Interaction flow (Sec. 4's working example) ----------------------
 * At fixed temperature T the flow parameter g scales the bare on-site
 * interaction (the propagator carries sqrt(g)); the one-loop equation for the
 * vertex then has the same three channels as the temperature flow with the
 * full bubble L_T in place of dL/dT:
 *   dV/dg = F_L[V],  F_L = the rhs of frg_rhs with B = binned w_p L(xi_p, xi2; T),
 *   Lpp = D[tanh](a, -b) / 4T,  Lph = D[tanh](a, b) / 4T  (a = xi_p / 2T,
 *   b = xi2 / 2T, D[f](x, y) = (f(x) - f(y)) / (x - y)).
 * The bubbles do not depend on g: a flow computes them once and every rhs is
 * the contraction alone.  The flow starts from V(g0) = V0 (V0 = U at g0 = 0:
 * the bare vertex; g V(g) is the effective interaction of the model whose
 * bare interaction is g U). */
typedef struct {
    frg_stepper stepper;
    frg_precision prec;
    double T;            /* fixed temperature (> 0) */
    double g0, g1;       /* flow range, g0 != g1 (0 -> 1 for the full interaction) */
    double rtol, atol, vmax, h0;
    int32_t fixed_steps, max_steps;
} frg_iflow_opts;

typedef struct {
    frg_stop reason;     /* FRG_STOP_TMIN: g1 reached */
    double g_end;        /* g of the final state */
    double g_c;          /* g at the first accepted step with max|V| > vmax (NaN if none) */
    double g_c_interp;   /* crossing interpolated linearly in g */
    int32_t accepted, rejected, rhs_evals, first_step_rhs;
} frg_iflow_result;

/* Full bubbles L_T (not their T-derivative) into d_bpp / d_bph, laid out as in
 * frg_bubbles (every row; FP64 or FP32 by prec).  Either output may be NULL. */
frg_status frg_bubbles_full(frg_ctx ctx, double T, frg_precision prec, void *d_bpp, void *d_bph,
                            void *stream);

/* One evaluation of F_L[V] = dV/dg at temperature T (bubbles and contraction;
 * the symmetry, zero-chunk and symmetric-vertex settings apply as in frg_rhs).
 * d_V and d_F are [N][N][N] FP64 and must not overlap. */
frg_status frg_rhs_full(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec,
                        void *stream);

/* Interaction flow, step by step: frg_iflow_init computes the bubbles L_T into
 * the context (they stay valid until another rhs, bubble or flow call on the
 * context) and initialises d_state (FRG_STATE_LEN doubles; FRG_ST_S holds g);
 * frg_iflow_step makes one step attempt on the device as frg_flow_step does
 * (EINVAL if the context's bubbles are no longer those of o->T). */
frg_status frg_iflow_init(frg_ctx ctx, const frg_iflow_opts *o, const double *d_V, double *d_state,
                          void *stream);
frg_status frg_iflow_step(frg_ctx ctx, const frg_iflow_opts *o, double *d_V, double *d_state,
                          void *stream);

/* Whole interaction flow from V0 (in d_V, overwritten with the final state);
 * the log rows are as in frg_flow with g in place of s. */
frg_status frg_iflow(frg_ctx ctx, const frg_iflow_opts *o, double *d_V, double *d_log, int32_t log_cap,
                     frg_iflow_result *r, void *stream);

/* Batches of independent flows (different model parameters, uneven N, the
 * same n_rad x n_ang).  Each flow keeps its own geometry and workspace; every
 * kernel of an RK stage runs once for the whole batch from work lists of
 * (flow, block).  The channel contraction of all flows is one launch per
 * block-height class over a work list sorted by cost, largest flows first,
 * which the hardware dispatcher deals out dynamically as compute units free up
 * (the dynamic schedule of Alg. 2 moved onto the device); setting
 * FRG_BATCH_DISPATCH=persistent uses persistent blocks pulling from per-XCD
 * queues through device counters instead.  Flows that have stopped are
 * skipped on the device.  Errors as for the single-flow calls. */
typedef struct frg_batch_s *frg_batch;
frg_status frg_batch_create(const frg_params *params, int32_t n_flows, frg_batch *out);
frg_status frg_batch_destroy(frg_batch b);
/* the context of flow i (owned by the batch; do not destroy) */
frg_status frg_batch_context(frg_batch b, int32_t i, frg_ctx *out);
/* F_i = dV_i/dT at T[i] (host array) for every flow; d_V, d_F: host arrays of
 * device pointers.  Synchronises the batch's internal stream. */
frg_status frg_batch_rhs(frg_batch b, const double *T, double *const *d_V, double *const *d_F,
                         frg_precision prec, void *stream);
/* DP5(4) flows of all members, one batched step (captured once in a hipGraph)
 * at a time, until every flow stopped.  d_log (nullable): [n_flows][log_cap][8]
 * as for frg_flow.  r: n_flows results. */
frg_status frg_batch_flow(frg_batch b, const frg_flow_opts *o, double *const *d_V, double *d_log,
                          int32_t log_cap, frg_flow_result *r, void *stream);
/* The same in pieces: initialise every member (first stage included), then
 * enqueue one batched step at a time (no synchronisation), then read the
 * members' results (synchronises; all_stopped nullable).  The V buffers must
 * stay valid until the flow is finished.  frg_batch_flow_step returns EINVAL
 * (and the batch needs frg_batch_flow_init again) if a member's workspace was
 * reallocated in between, e.g. by an rhs on its context in another mode. */
frg_status frg_batch_flow_init(frg_batch b, const frg_flow_opts *o, double *const *d_V, double *d_log,
                               int32_t log_cap, void *stream);
frg_status frg_batch_flow_step(frg_batch b, void *stream);
frg_status frg_batch_results(frg_batch b, frg_flow_result *r, int32_t *all_stopped);

/* C4v reduction of the bubble work (Sec. 4 counts independent couplings after
 * using the lattice symmetries): for N % 8 == 0 the grid is bitwise C4v
 * symmetric, B_{g t}(g a, g b) = B_t(a, b), and each rhs evaluates the bubble
 * rows of one transfer per orbit only (about 1/8 of them); the contraction
 * reads the other rows through the patch permutation.  frg_create enables it
 * after checking the relation exactly on the second-line patch table (setting
 * FRG_NO_SYM in the environment leaves it off).  frg_set_symmetry switches it
 * (ENOTSUP when unavailable); frg_symmetry reports whether it is on and how
 * many bubble rows one rhs computes. */
frg_status frg_set_symmetry(frg_ctx ctx, int32_t enable);
frg_status frg_symmetry(frg_ctx ctx, int32_t *active, int32_t *rows_computed);

/* Zero-block skipping in the channel contractions (Sec. 4's one-loop diagrams
 * integrated over the Brillouin zone on N patches: here the sums over the loop
 * patch pair (a, b) of a bubble row).  The entry (a, b) of
 * a bubble row is a sum over the fine points of patch a whose second momentum
 * lies in patch b, so it is exactly zero whenever there is no such point; the
 * pattern is fixed by the patch geometry, independent of T.  frg_create orders
 * the contraction columns along a Hilbert curve of their transfer momentum and
 * lists, per tile of 64 columns, the 8-wide k chunks (k = a*N + b) where any
 * of the tile's rows has a point; the contraction then visits only those.
 * Skipped terms are exact zeros, so the result changes only by the order of
 * the FP sums.  frg_set_kskip(ctx, 0) switches to the dense contraction
 * (natural column order, every chunk; allocates its lists on first use);
 * frg_kskip reports whether skipping is on and the executed share of the
 * dense multiply-adds (channels weighted pp 1, phc 1, phd 2).  Batches made
 * by frg_batch_create always skip. */
frg_status frg_set_kskip(frg_ctx ctx, int32_t enable);
frg_status frg_kskip(frg_ctx ctx, int32_t *active, double *executed_frac);

/* Symmetric-vertex mode (Sec. 4: the independent couplings are counted after
 * using the lattice symmetries).  For a vertex that is invariant under the
 * C4v point group, V(g k1, g k2, g k3) = V(k1, k2, k3), the rhs is invariant
 * too, and with the exactly covariant grid (N % 8 == 0) the contraction needs
 * one output column per C4v orbit of column pairs (about N^2/8 of them,
 * i.e. about N^3/8 independent entries); the combine writes every entry of F
 * from them.  frg_set_vsym(ctx, 1) asserts that every V passed to frg_rhs
 * is invariant (not checked there); frg_flow_init checks V0 (relative
 * deviation at most 1e-12, else FRG_EINVAL), and a flow from an invariant V0
 * stays invariant.  ENOTSUP when N % 8 != 0 or the covariance check at
 * creation failed.  frg_vsym reports the mode and the columns computed per
 * channel.  frg_check_vsym computes max_{g,j} |V(g j) - V(j)| / max |V| for a
 * device V (synchronises the stream).  frg_batch_set_vsym sets the mode for
 * every flow of a batch; the batch must be flow_init'ed again afterwards.
 * With a self-energy flowing along the mode needs it C4v invariant
 * (frg_set_self_energy value 2; EINVAL with a general one). */
frg_status frg_set_vsym(frg_ctx ctx, int32_t enable);
frg_status frg_vsym(frg_ctx ctx, int32_t *active, int32_t *columns);
frg_status frg_check_vsym(frg_ctx ctx, const double *d_V, double *rel_dev, void *stream);
frg_status frg_batch_set_vsym(frg_batch b, int32_t enable);

/* Kernel timing with HIP events recorded on the launch stream around every
 * kernel of the rhs and flow pipelines (for measurement; off by default).
 * frg_profile_begin clears and enables the record; frg_profile_end
 * synchronises the recorded events, writes per kernel class the summed
 * milliseconds and launch counts (arrays of FRG_KERNEL_CLASSES entries; either
 * may be NULL) and disables recording. */
enum {
    FRG_K_PREP = 0, FRG_K_BUBBLES = 1, FRG_K_LAYOUT = 2, FRG_K_CONTRACT = 3,
    FRG_K_COMBINE = 4, FRG_K_RK = 5, FRG_KERNEL_CLASSES = 6
};
frg_status frg_profile_begin(frg_ctx ctx);
frg_status frg_profile_end(frg_ctx ctx, double *ms, int32_t *counts);
/* ---- Tuning (tile shapes and work granularity picked by measurement; the
 * paper's load-balancing lessons, Alg. 2 and Sec. 6, are about the same
 * granularity choices).  Three launch parameters of the rhs:
 *   kparts      K parts the channel contraction is cut into for the column set
 *               in use (every column / one per C4v orbit / dense), 1..64;
 *   sweep_rows  bubble rows per block of the sweep, a multiple of 4 in 4..256
 *               (single flows; for a batch, rows per block of the batched sweep);
 *   block_rows  output rows per contraction block: 32, 64 or 96.
 * A 0 field in frg_set_tuning keeps the current value.  Results do not change
 * bit for bit with kparts (the K-part sums round differently) but stay within
 * the bars of the rhs; nothing else changes the arithmetic.  frg_set_tuning
 * drops a captured step; a batch needs frg_batch_flow_init again. */
typedef struct {
    int32_t kparts, sweep_rows, block_rows;
} frg_tuning;
frg_status frg_get_tuning(frg_ctx ctx, frg_tuning *t);
frg_status frg_set_tuning(frg_ctx ctx, const frg_tuning *t);
/* Autotuner: times the rhs at T on d_V (into d_F, caller's device buffers) in
 * the context's current mode and precision with HIP events, reps evaluations
 * per candidate after a warm-up one: first the sweep's rows per block against
 * the bubble kernels' time, then (block_rows, kparts) against the contraction
 * and K-part sum time; applies the best and returns it with its per-rhs kernel
 * time in ms (best, best_ms nullable).  log (host, nullable): up to log_cap rows
 * of 6 doubles per candidate (kparts, sweep_rows, block_rows, then ms per rhs of
 * the bubbles, of the contraction and K-part sum, of all kernels); *log_rows
 * (nullable) receives the number of candidates.  Synchronises. */
frg_status frg_tune(frg_ctx ctx, double T, const double *d_V, double *d_F, frg_precision prec, int32_t reps,
                    frg_tuning *best, double *best_ms, double *log, int32_t log_cap, int32_t *log_rows,
                    void *stream);
/* The same for a batch: every member takes each candidate, the batched rhs of
 * all flows (T[i], d_V[i] -> d_F[i]) is timed; frg_batch_set_tuning applies one
 * tuning to every member.  Both require frg_batch_flow_init again before steps. */
frg_status frg_batch_set_tuning(frg_batch b, const frg_tuning *t);
frg_status frg_batch_tune(frg_batch b, const double *T, double *const *d_V, double *const *d_F,
                          frg_precision prec, int32_t reps, frg_tuning *best, double *best_ms, double *log,
                          int32_t log_cap, int32_t *log_rows, void *stream);

/* The same for the batched kernels of a batch (one launch per class covers
 * every flow); while it is on, frg_batch_flow_step launches eagerly instead of
 * replaying its captured step, so that events sit between the kernels. */
frg_status frg_batch_profile_begin(frg_batch b);
frg_status frg_batch_profile_end(frg_batch b, double *ms, int32_t *counts);

const char *frg_status_str(frg_status st);
const char *frg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

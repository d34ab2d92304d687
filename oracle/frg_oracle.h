/*
 * frg_oracle.h -- plain FP64 CPU oracle for the one-loop temperature-flow
 * right-hand side of the 2D Hubbard four-point vertex on N momentum patches.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * Paper anchors (Rohe, "Hierarchical Parallelisation of Functional
 * Renormalisation Group Calculations - hp-fRG"):
 *   - Sec. 2, Eq. (1): the discretised flow dV[i]/dg = F[V[j]; g] over one
 *     flat array of couplings, integrated with an explicit stepper so that F
 *     is evaluated with V frozen.
 *   - Sec. 4: 2D square-lattice Hubbard model with hoppings t, t' and chemical
 *     potential mu; three one-loop diagrams (particle-particle, direct and
 *     crossed particle-hole) integrated over the Brillouin zone; N patches.
 * The concrete formulas (patch geometry, bubble integrands, signs of the three
 * channels, flow in s = ln T) are the readings listed at the top of the design
 * notes; each function below states which one it implements.
 */
#ifndef FRG_ORACLE_H
#define FRG_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_model orc_model;

/* Model parameters: dispersion eps(k) = -2t(cos kx + cos ky) - 4t' cos kx cos ky - mu,
 * bare on-site U (initial condition V = U), N patches (N % 4 == 0, 4 <= N <= 256),
 * n_rad x n_ang fine loop points per patch. */
typedef struct {
    double t, tp, mu, U;
    int32_t N, n_rad, n_ang;
} orc_params;

/* Build the geometry (patch centres, sector boundaries, fine grid, transfer
 * momenta).  Returns NULL on invalid parameters. */
orc_model *orc_create(const orc_params *p);

/* The same with the paper's quadrature as the fine grid (Sec. 4): n_E
 * equidistant energy midpoints across the band, and along each energy, per
 * patch sector, a locally adaptive trisection midpoint rule in the angle of the
 * ray from Gamma (relative target rtol of the shell's inner integral, at most
 * 3^max_level points per sector and shell).  The weights are those of the
 * quadrature (not normalised).  Every patch holds nf points (orc_nf), padded
 * with zero-weight points; p->n_rad, p->n_ang are ignored (the model reports
 * 1 and nf).  NULL on invalid parameters or |t'| >= t/2. */
typedef struct {
    int32_t n_E, max_level;
    double rtol;
} orc_egrid;
orc_model *orc_create_egrid(const orc_params *p, const orc_egrid *e);
void orc_destroy(orc_model *m);
void orc_set_threads(int n);          /* OpenMP threads used by the heavy loops */
int orc_get_threads(void);

/* sizes */
int32_t orc_N(const orc_model *m);
int32_t orc_nf(const orc_model *m);
int32_t orc_num_pp(const orc_model *m);   /* N(N+1)/2 */
int32_t orc_num_ph(const orc_model *m);   /* N(N-1)+1 */

/* Geometry export (any pointer may be NULL):
 *   kc[N][2], bnd[(N+1)][2], fine[N*n_f][4] = (px, py, w, xi),
 *   qpp[Tpp][2], qph[Tph][2], idx4[N][N][N] = patch of k1+k2-k3. */
void orc_tables(const orc_model *m, double *kc, double *bnd, double *fine,
                double *qpp, double *qph, int32_t *idx4);
/* row index of the pp transfer of (j1,j2) and of the ph transfer Q = k_x - k_y */
int32_t orc_row_pp(const orc_model *m, int32_t j1, int32_t j2);
int32_t orc_row_ph(const orc_model *m, int32_t x, int32_t y);

/* primitive maps */
double orc_eps(const orc_model *m, double kx, double ky);
double orc_fold(double x);                                  /* into [-pi, pi) */
int32_t orc_project(const orc_model *m, double kx, double ky);  /* folds, then sector */

/* Bubble integrands (kind 0 = particle-hole, 1 = particle-particle).
 * deriv = 0: L(xi1, xi2; T); deriv = 1: dL/dT. */
double orc_L(int32_t kind, int32_t deriv, double xi1, double xi2, double T);

/* second-line patch of every (transfer row, fine point): out[T][N*n_f] */
void orc_bins(const orc_model *m, int32_t kind, int32_t *out);

/* Binned bubble tensors Bpp[Tpp][N][N], Bph[Tph][N][N] (either may be NULL). */
void orc_bubbles(const orc_model *m, double T, int32_t deriv, double *Bpp, double *Bph);

/* rhs F = dV/dT for all N^3 entries through the binned bubble tensors. */
void orc_rhs(const orc_model *m, double T, const double *V, double *F);
/* Same contraction with caller-supplied bubble tensors (deriv or not). */
void orc_contract(const orc_model *m, const double *Bpp, const double *Bph,
                  const double *V, double *F);
/* Brute force: selected entries by a direct fine-grid sum, no bubble tensors. */
void orc_rhs_entries(const orc_model *m, double T, const double *V, int64_t n,
                     const int32_t *j123, double *out);

/* Self-energy (a static value S_j per patch flowing with the vertex; S may be
 * NULL for zero).  Every loop line carries its own patch's S:
 * L(xi_p + S_a, eps(second line) + S_b).
 *   orc_bubbles_se: the bubble tensors with S;
 *   orc_dsigma: dS_j/dT = sum_a D_a [2 V(j,a,j) - V(a,j,j)],
 *               D_a = sum_{p in a} w_p d/dT n_F((xi_p + S_a)/T) at fixed S;
 *   orc_rhs_se: F (as orc_rhs, with S in the bubbles) and dS;
 *   orc_rhs_entries_se: brute-force F entries with S. */
void orc_bubbles_se(const orc_model *m, double T, int32_t deriv, const double *S, double *Bpp, double *Bph);
void orc_dsigma(const orc_model *m, double T, const double *V, const double *S, double *dS);
void orc_rhs_se(const orc_model *m, double T, const double *V, const double *S, double *F, double *dS);
void orc_rhs_entries_se(const orc_model *m, double T, const double *V, const double *S, int64_t n,
                        const int32_t *j123, double *out);

/* Generic explicit steppers in s for dy/ds = f(s, y). */
typedef void (*orc_ode_fn)(void *ctx, double s, const double *y, double *dyds, int64_t n);

enum { ORC_STOP_NONE = 0, ORC_STOP_TMIN = 1, ORC_STOP_DIVERGED = 2,
       ORC_STOP_MAXSTEPS = 3, ORC_STOP_NONFINITE = 4, ORC_STOP_HMIN = 5 };

typedef struct {
    int32_t reason;
    double s_end;          /* final flow variable */
    double s_c;            /* s at the first accepted step with max|y| > vmax (else NaN) */
    double s_c_interp;     /* crossing interpolated linearly in s */
    int32_t accepted, rejected, rhs_evals;
    int32_t first_step_rhs;   /* rhs evaluations spent on the first accepted step */
} orc_ode_result;

/* classical RK4 with nsteps uniform steps from s0 to s1; stops after a step
 * whose max|y| exceeds vmax (divergence is a result, not an error) */
int32_t orc_rk4(orc_ode_fn f, void *ctx, int64_t n, double *y, double s0, double s1,
                int32_t nsteps, double vmax, orc_ode_result *r);
/* Dormand-Prince 5(4) with FSAL and the step control of the design notes.
 * log (nullable) receives per accepted step: s, h_used, err, max|y|, rhs_evals, rejected. */
int32_t orc_dp54(orc_ode_fn f, void *ctx, int64_t n, double *y, double s0, double s_min,
                 double h0, double rtol, double atol, double vmax, int32_t max_steps,
                 orc_ode_result *r, double *logbuf, int32_t log_cap);

/* The fRG temperature flow: dV/ds = T F(V, T), s = ln T, from T0 down.
 * stepper 0 = RK4 with fixed_steps log-spaced steps to T_min (vmax stop),
 * stepper 1 = DP5(4) with rtol/atol/vmax/h0/max_steps. */
typedef struct {
    int32_t stepper;
    double T0, T_min, rtol, atol, vmax, h0;
    int32_t fixed_steps, max_steps;
} orc_flow_opts;
int32_t orc_flow(const orc_model *m, const orc_flow_opts *o, double *V, orc_ode_result *r,
                 double *logbuf, int32_t log_cap);

#ifdef __cplusplus
}
#endif
#endif

// Internal declarations of libfrg: host geometry, context, kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/frg.h"

namespace frg {

// ----------------------------------------------------------------- geometry
// Host-side patch geometry in plain FP64 (built with -ffp-contract=off so
// every product and sum is rounded exactly as written).
struct Geometry {
    int N = 0, n_rad = 0, n_ang = 0, nf = 0, np = 0, Tpp = 0, Tph = 0;
    double t = 0, tp = 0, mu = 0, U = 0, dth = 0;
    // energy-angle grid: each patch's live points first, then zero-weight
    // padding up to nf (a multiple of kSegPoints); count[a] live points
    bool egrid = false;
    std::vector<int32_t> count;           // [N], egrid only
    std::vector<double> kc, bnd;          // [N][2], [N+1][2]
    std::vector<double> px, py, w, xi;    // [np]
    std::vector<double> qpp, qph;         // [Tpp][2], [Tph][2]
    std::vector<int32_t> row_pp, row_ph;  // [N][N]: (j1,j2) -> pp row, (x,y) -> ph row
};

void build_geometry(const frg_params &p, Geometry &g);
// points per segment of the energy-angle sweep; the padded n_f is a multiple
constexpr int kSegPoints = 512;
// the energy-angle quadrature (frg_create_egrid) as the fine grid; false when
// the points of a patch exceed max_nf
bool build_geometry_egrid(const frg_params &p, const frg_egrid &e, int max_nf, Geometry &g);
double fold_bz(double x);
int32_t host_patch(const Geometry &g, double kx, double ky);
void host_idx4(const Geometry &g, int32_t *out);

// ----------------------------------------------------------------- launchers
// second-line patch of every (row, point); rows: pp rows then ph rows.  Within
// a row each patch's points are stored angular-fastest: fine point (s, m) of
// patch a (fine-grid index a*n_f + s*n_rad + m) at a*n_f + m*n_ang + s
void launch_bins(const double *bnd, const double *px, const double *py, const double *qrow,
                 int N, int n_rad, int n_ang, int Tpp, int Trows, uint8_t *bins, hipStream_t s);
// rows r0 .. r0 + nrows - 1 of the table copied out in fine-grid order
void launch_bins_export(const uint8_t *bins, int N, int n_rad, int n_ang, int r0, int nrows, uint8_t *out,
                        hipStream_t s);

// per-point temperature-dependent factors (a = xi/2T, h(a), -w/4T^2); T is
// either T_host, or exp(state[s] + c*state[h]) when state != nullptr
void launch_point_prep(const double *xi, const double *w, int np, double T_host,
                       const double *state, double c_stage, double *pa64, float *pa32,
                       double *Tout, hipStream_t s, const double *sigma = nullptr, int nf = 1);

// self-energy flow (one value per patch): D[a] = sum_{p in a} w_p d/dT n_F((xi_p + S_a)/T)
// (one block per patch, fixed-order sums), then
// dS[j] = scale * sum_a D[a] (2 V(j,a,j) - V(a,j,j)), scale = T when scale_by_T;
// V a full vertex, or a reduced flow state when ppos (the pp column map) is given
void launch_dsigma(const double *xi, const double *w, int N, int nf, const double *V, const double *S,
                   const double *Tdev, int scale_by_T, double *D, double *dS, hipStream_t s,
                   const int32_t *ppos = nullptr);

struct BubbleArgs {
    int N, nf, np, Tpp, Trows;
    int n_rad, n_ang;              // fine grid of a patch (n_f = n_rad * n_ang)
    double mt2, mt4p, mu;          // -2t, 4t', mu
    const uint8_t *bins;           // [Trows][np], patches' points angular-fastest
    const double *trig_row;        // [Trows][4]: cos qx, sin qx, cos qy, sin qy
    const double *trig_pt;         // [4][np]: cos px, sin px, cos py, sin py
    const double *pa64;            // [3][np]: a, h(a), -w/4T^2   (FP64 path)
    const float *pa32;             // [3][np]                      (split path)
    const double *Tdev;            // [0] = T
    void *Bpp, *Bph;               // outputs (double or float)
    // rows to compute: output position o < nrows evaluates transfer row
    // rowlist[o] (or o itself when rowlist == nullptr); positions below
    // npp_out go to Bpp, the rest to Bph
    int nrows, npp_out;
    const int32_t *rowlist;
    // pairs: when set, position o evaluates the pp row rowlist[o] into Bpp and
    // the ph row rowlist_ph[o] (the opposite transfer) into Bph, both at o
    const int32_t *rowlist_ph;
    int rpb;   // rows per block of the sweep (a multiple of 4, at most 256; 0: the single-flow default)
    // energy-angle grid: live points of each patch ([N]); the sweep then walks
    // them in segments of kSegPoints (nullptr: polar grid, n_f <= 1024)
    const int32_t *count;
    // self-energy per patch ([N], nullptr: none): the second line's energy
    // carries S of its patch (the first line's is in pa); dL/dT rows, paired
    // only when S is C4v invariant
    const double *sigma;
};
// full: the bubble L itself (interaction flow) instead of dL/dT
void launch_bubbles(const BubbleArgs &a, bool fp32, bool full, hipStream_t s);

// verify the pair identity of the second-line table: at every point the ph row
// of -q has the pp row q's patch + N/2 (counts the mismatches)
void launch_pair_check(const uint8_t *bins, const int32_t *rows_pp, const int32_t *rows_ph, int npairs, int np,
                       int N, int *mismatch, hipStream_t s);

// verify B_{g t}(g a, g b) = B_t(a, b) on the second-line table: counts the
// (row, point) entries where bins[t'][p'] != g(bins[rep(t')][g^-1 p'])
void launch_sym_check(const uint8_t *bins, const int32_t *orbit, int N, int n_rad, int n_ang,
                      int Trows, bool rev, int *mismatch, hipStream_t s);

// permuted copies of V used as contraction operands (FP64)
void launch_layout_f64(const double *V, int N, double *perm, hipStream_t s);
// split-BF16 operands: hi/lo of the four A matrices + FP32 gather tables
void launch_layout_split(const double *V, int N, uint16_t *ahl, float *g32, hipStream_t s);
int layout_blocks(int N);   // blocks (of 256 threads) of one layout pass

enum Term { TERM_PP = 0, TERM_PHC = 1, TERM_PHD = 2 };

// all three channels in one launch; term t writes C[t] + part * n3 for K part
// `part`, laid out [tile position p][m] (p holds column cperm[t][p])
struct FusedContractArgs {
    int N, KS, mtiles, ctiles;
    int bm;            // output rows per block: 32, 64 or 96 (0: by N)
    int64_t pstride;   // elements between K parts of a term's partials (computed columns x N)
    int fast;   // split path: buffer-load fast path (N % 32 == 0, bubble rows < 2 GiB)
    int ncol[3];  // columns computed per term (N^2, or one per C4v orbit of column pairs)
    int64_t n3;
    const void *B[3];             // bubble rows per term (pp: Bpp, phc/phd: Bph)
    int64_t Bbytes[3];            // their sizes in bytes
    // column c -> (stored row << 3) | o: the column's bubble row is the stored
    // row acted on by C4v element o, B_col(a', b') = B_stored(o^-1 a', o^-1 b')
    const int32_t *colrow[3];
    // column tiles: tile position -> column (columns ordered so that a tile's
    // transfers are close in k space), and per tile the list of 8-wide k
    // chunks that hold a structural nonzero of any of its bubble rows
    // in increasing order; K part ks of tile t is klist[koff[t*(KS+1)+ks] ..
    // koff[t*(KS+1)+ks+1]), KS being the value the offsets were cut for; an entry packs the
    // chunk id j and the patch pair (a, b) of k = 8j = a*N + b as
    // j | a << 13 | b << 21)
    const int32_t *cperm[3];
    const int32_t *koff[3];
    const int32_t *klist[3];
    const double *A64[3][2];
    const uint16_t *Ahl[3][2];
    const double *G64[3][2];
    const float *G32[3][2];
    void *C[3];   // partials [KS][pstride]: float in the split path, double in the FP64 path
};
void launch_contract_fused(const FusedContractArgs &a, bool split, hipStream_t s);
int contract_block_rows(int N);
// block kinds of one (m tile, column tile, K part), heaviest first, and the
// number of products each multiplies: {phd: 2, phc: 1, pp: 1} in both paths
int contract_kinds(bool split);
int contract_kind_products(bool split, int kind);
constexpr int kContractCols = 64;     // columns per contraction tile
constexpr int kContractChunk = 8;     // k chunk of the active lists
// flags[t][j] = 1 if some column at tile position t*64 .. t*64+63 (< ncol) has
// a point of the second-line table in k chunk j (k = a*N + b, chunk = k / 8);
// colfull[c] is the full row (pp rows, then ph rows) of column c; flags must be
// zeroed by the caller (only ones are written)
void launch_tile_pattern(const uint8_t *bins, const int32_t *colfull, const int32_t *cperm, int ncol, int N,
                         int nf, int np, uint8_t *flags, hipStream_t s);

// F[j1][j2][j3] = scale * (-Cpp(j1,j2; j3) + Cc(j2,j3; j1) + Cd(j1,j3; j2)), each
// channel summed (in FP64) over the K parts.  Channel value C(c; m) of column c
// (pp: j1*N+j2, ph: y*N+x) and free index m is C[pos][perm8[h][m]] with
// cmap[c] = (pos << 3) | h: pos the tile position of the computed column, h
// the C4v element that carries c's frame to it (0 when every column is
// computed; perm8 = [8][N] patch maps).  scale = T when scale_by_T; the
// partials are float when f32parts, else double
void launch_combine(const void *Cpp, const void *Cc, const void *Cd, bool f32parts, int N, int parts,
                    const int32_t *ppos, const int32_t *phpos, const int16_t *perm8, const double *Tdev,
                    int scale_by_T, double *F, hipStream_t s);
// largest |V(g j1, g j2, g j3) - V(j1, j2, j3)| over the C4v elements g, and
// max |V|: per-block partials [2][nblocks] (host reduces)
int vsym_check_blocks(int N);
void launch_vsym_check(const double *V, int N, const int16_t *perm8, double *partials, hipStream_t s);
int combine_tiles(int N);   // blocks of one combine
// out[t][i] = sum_ks C_t[ks][i] in FP64 for the three channels t and i < nel,
// where C_t starts at double offset t*KS*cs of C and holds float (f32parts)
// or double partials (part stride cs); out is [3][cs]
void launch_sum_parts(const double *C, bool f32parts, int KS, int64_t cs, int64_t nel, double *out,
                      hipStream_t s);
constexpr int kSumPartsPerBlock = 1024;   // elements of out per block of the batched sum

// ----------------------------------------------------------------- RK kernels
struct RkStageArgs {
    int64_t n;
    const double *y;
    const double *k[7];
    double coef[7];
    int nk;
    const double *state;   // h = state[FRG_ST_H]
    double *out;
};
void launch_rk_stage(const RkStageArgs &a, hipStream_t s);
// DP5(4) error norm + max|y5|: partials then final (deterministic max)
void launch_dp_error(int64_t n, const double *y, const double *y5, const double *const k[7],
                     const double e[7], double rtol, double atol, double *state, double *partial,
                     int nblocks, hipStream_t s);
void launch_maxabs_to(int64_t n, const double *y, double *state, int slot, double *partial,
                      int nblocks, hipStream_t s);
void launch_state_set(double *state, int slot, double v, hipStream_t s);
void launch_pre_step(double *state, int stepper, hipStream_t s);
void launch_dp_control(double *state, double *log, int log_cap, double vmax, int max_steps,
                       int stepper, hipStream_t s);
// split layout straight from a reduced state (gather rows of representative columns only)
void launch_layout_split_red(const double *Vr, int N, const int32_t *ppos, const int32_t *cperm_ph, int ncol_ph,
                             uint16_t *ahl, float *g32, hipStream_t s);
// Reduced flow state of the symmetric-vertex mode (entry pos * N + m = V(cperm[pos], m)):
// gather it from a full V, expand it into a full V (only accepted steps when gate,
// the flow state, is given), and the rhs at the representative entries only.
void launch_vred_gather(const double *V, int N, const int32_t *cperm, int64_t nst, double *Vr, hipStream_t s);
void launch_vred_expand(const double *Vr, int N, const int32_t *cmap, const int16_t *perm8, const double *gate,
                        double *V, hipStream_t s);
void launch_combine_red(const double *Cs, int64_t cs, int N, int64_t nst, const int32_t *cperm,
                        const int32_t *phpos, const int16_t *perm8, const double *Tdev, int scale_by_T, double *F,
                        hipStream_t s);
// dst <- src when the flow state says the step was accepted (state null: always)
void launch_accept_copy(int64_t n, const double *state, const double *src, double *dst,
                        hipStream_t s);
void launch_state_init(double *state, double s0, double h, double s_min, hipStream_t s);

// ----------------------------------------------------------------- batches
// Per-flow pointers used by the batched launches (one entry per flow, in
// device memory); work lists are arrays of (flow, local block).
struct FlowArgs {
    int N, np, nred;
    int64_t n3;
    const double *xi, *w;
    double *pa64;
    float *pa32;
    double *Tdev;
    double *V, *state;
    double *k[7];
    double *yt, *y5, *partial;
    double *perm;
    uint16_t *ahl;
    float *g32;
    double *C;   // [3][KS][cs] doubles; the split path keeps float partials in it
    int KS;
    int f32parts;  // partials are float (split path)
    int64_t cs;    // channel stride: elements computed per channel (ncol * N)
    double *Csum;  // [3][cs]: partials summed over the K parts
    int64_t nel;   // elements per channel actually computed (ncol * N)
    const int16_t *perm8;   // [8][N] C4v patch maps
    const int32_t *ppos, *phpos;   // tile position of each pp / ph column
    // reduced state (symmetric-vertex mode with orbit columns): the stage vectors
    // k, yr, ytr, y5r hold nst = ncol_pp * N entries (pp representative columns
    // cperm_pp in tile order); yt and y5 then hold the full rhs inputs
    int red;
    int64_t nst;
    double *yr, *ytr, *y5r;
    const int32_t *cperm_pp;
    const int32_t *cperm_ph;   // representative ph columns (the layout's phc gather rows)
    int ncol_ph;
};
enum { SRC_V = 0, SRC_YT = 1, SRC_Y5 = 2 };
// batched: dst SRC_V gathers yr from V (items over the reduced length), SRC_YT /
// SRC_Y5 expand ytr / y5r into yt / y5 (items over n3); other flows skip
void launch_vred_b(const FlowArgs *fa, const int2 *items, int nitems, int dst, hipStream_t s);

// rows per block of the batched sweep for nrows rows (its items are (flow, chunk << 8 | patch))
int bubble_batched_rows_per_block(int nrows);
// items: the first npaired belong to flows with row pairs (rowlist_ph set)
void launch_bubbles_batched(const BubbleArgs *args, const int2 *items, int npaired, int nitems,
                            const double *const *states, int nf, int maxN, bool fp32, hipStream_t s);
size_t contract_lds_bytes(bool split);
void launch_contract_items(const FusedContractArgs *args, const int2 *items, int nitems,
                           const double *const *states, int bm, bool split, hipStream_t s);
void launch_contract_persistent(const FusedContractArgs *args, const int2 *items, const int *qstart,
                                const int *qcount, int *counters, const double *const *states, int grid,
                                int bm, bool split, hipStream_t s);
void launch_prep_b(const FlowArgs *fa, const int2 *items, int nitems, double c_stage, bool split,
                   hipStream_t s);
// items: (flow, block < layout_blocks(N) of the flow)
void launch_layout_b(const FlowArgs *fa, const int2 *items, int nitems, int src, bool split,
                     hipStream_t s);
void launch_combine_b(const FlowArgs *fa, const int2 *items, int nitems, int stage, hipStream_t s);
void launch_sum_parts_b(const FlowArgs *fa, const int2 *items, int nitems, hipStream_t s);
void launch_rk_stage_b(const FlowArgs *fa, const int2 *items, int nitems, const double coef[7],
                       int nk, int dst, hipStream_t s);
void launch_dp_error_b(const FlowArgs *fa, const int2 *items, int nitems, int nflows,
                       const double e[7], double rtol, double atol, hipStream_t s);
void launch_step_ctl_b(const FlowArgs *fa, int nflows, int phase, double *log_base, int log_cap,
                       double vmax, int max_steps, hipStream_t s);
void launch_accept_b(const FlowArgs *fa, const int2 *items, int nitems, hipStream_t s);

// ----------------------------------------------------------------- static scratch
// bytes of the library's static device scratch (frg_rhs_noalloc)
constexpr size_t kScratchBytes = FRG_NOALLOC_SCRATCH_BYTES;
// device address of the scratch on the current device (looked up once per
// device; host code passes this, never the array's own name)
hipError_t scratch_address(void **out);

}  // namespace frg

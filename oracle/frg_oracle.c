/*
 * frg_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * What it computes: the right-hand side F = dV/dT of the one-loop temperature
 * flow of the static SU(2) four-point vertex V(k1,k2,k3) of the 2D
 * square-lattice Hubbard model on N patches, and explicit RK4 / DP5(4) flows
 * of Eq. (1) (Sec. 2) in s = ln T.  Everything is plain loops in double
 * precision; nothing is blocked, fused or reordered beyond the definitions.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library; the GPU library shares no code with it.
 *
 * Readings of the paper used here (the paper states the problem in prose:
 * Sec. 2 and Sec. 4 name the model, the three one-loop diagrams, the 2D
 * Brillouin-zone quadrature and the patch discretisation; it prints neither
 * formulas nor the patch geometry):
 *   G1 dispersion, G2 patches, G3 fine grid, G4 bubble integrands,
 *   G5 loop lines, G6 projection, G7 vertex, G8 rhs, G9 flow variable,
 *   G10 DP5(4) control -- spelled out next to each function.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-builtin-sin -fno-builtin-cos
 * -fPIC -shared (no fast-math), so every floating-point operation is the one
 * written and every sin and cos is its own libm call (gcc would otherwise merge
 * a sin and a cos of one argument into one sincos call, whose last bit can
 * differ from theirs).
 */
#include "frg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
static const double PI_D = ORC_PI;            /* double nearest pi */
static const double TWO_PI_D = 2.0 * ORC_PI;  /* exactly twice PI_D */

struct orc_model {
    orc_params p;
    int N, nf, Tpp, Tph;
    int egrid;             /* 1: energy-angle fine grid (eg_* below), 0: polar grid */
    double *eg_pts;        /* [patches built][nf][3] x, y, w of the energy-angle grid */
    double dth;            /* sector width 2 pi / N */
    double *kc;            /* [N][2] patch centres */
    double *bnd;           /* [N+1][2] sector boundary directions */
    double *px, *py, *w, *xi; /* [N*nf] fine grid: point, weight, energy */
    double *qpp, *qph;     /* [T][2] transfer momenta */
    int32_t *rpp, *rph;    /* [N][N] row maps */
};

static int g_threads = 0;
void orc_set_threads(int n) { g_threads = n; }
int orc_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}
#define NT orc_get_threads()

/* ------------------------------------------------------------------ G1 */
/* eps(k) = -2t (cos kx + cos ky) - 4t' cos kx cos ky - mu.  With t'=-0.01,
 * mu=-0.02 (Sec. 4) eps(pi,0) = 4t'-mu < 0, so the Fermi surface closes
 * around (pi,pi) as the paper states.  The product cx*cy is formed first so
 * that eps(x,y) == eps(y,x) bit for bit. */
static double eps_k(const orc_params *p, double kx, double ky)
{
    double cx = cos(kx), cy = cos(ky);
    return (-2.0 * p->t) * (cx + cy) - (4.0 * p->tp) * (cx * cy) - p->mu;
}
double orc_eps(const orc_model *m, double kx, double ky) { return eps_k(&m->p, kx, ky); }

/* ------------------------------------------------------------------ G6 fold */
double orc_fold(double x)
{
    while (x >= PI_D) x -= TWO_PI_D;
    while (x < -PI_D) x += TWO_PI_D;
    return x;
}

/* C4v element o (0..7) applied to (x, y); exact (swap / negate only). */
static void c4v(int o, double x, double y, double *ox, double *oy)
{
    switch (o) {
    case 0: *ox = x;  *oy = y;  break;
    case 1: *ox = y;  *oy = x;  break;
    case 2: *ox = -y; *oy = x;  break;
    case 3: *ox = -x; *oy = y;  break;
    case 4: *ox = -x; *oy = -y; break;
    case 5: *ox = -y; *oy = -x; break;
    case 6: *ox = y;  *oy = -x; break;
    default: *ox = x; *oy = -y; break;
    }
}

/* ------------------------------------------------------------------ G2 */
/* Distance from Gamma to the zone edge along direction (c, s). */
static double ray_extent(double c, double s)
{
    double ac = fabs(c), as = fabs(s);
    return PI_D / (ac > as ? ac : as);
}

/* Fermi-surface crossing along the ray: first sign change of eps over 1024
 * uniform nodes in (0, R], bisected 100 times; otherwise the node of least
 * |eps| (lowest index on ties). */
static double ray_root(const orc_params *p, double c, double s, double R)
{
    double rprev = R * 1.0 / 1024.0;
    double eprev = eps_k(p, rprev * c, rprev * s);
    double best_r = rprev, best_e = fabs(eprev);
    for (int i = 2; i <= 1024; i++) {
        double r = R * (double)i / 1024.0;
        double e = eps_k(p, r * c, r * s);
        if ((e >= 0.0) != (eprev >= 0.0)) {
            double lo = rprev, hi = r;
            int plo = (eprev >= 0.0);
            for (int it = 0; it < 100; it++) {
                double mid = 0.5 * (lo + hi);
                if ((eps_k(p, mid * c, mid * s) >= 0.0) == plo) lo = mid;
                else hi = mid;
            }
            return 0.5 * (lo + hi);
        }
        if (fabs(e) < best_e) { best_e = fabs(e); best_r = r; }
        rprev = r;
        eprev = e;
    }
    return best_r;
}

/* ------------------------------------------------------------------ G6 project */
static double cross2(const double *b, double kx, double ky)
{
    double u = b[0] * ky;
    double v = b[1] * kx;
    return u - v;
}

static int in_sector(const orc_model *m, int j, double kx, double ky)
{
    return cross2(m->bnd + 2 * j, kx, ky) >= 0.0 && cross2(m->bnd + 2 * (j + 1), kx, ky) < 0.0;
}

/* pi(k): fold both components into [-pi, pi), then the unique sector j with
 * cross(b_j, k) >= 0 and cross(b_{j+1}, k) < 0 (half-open, counter-clockwise
 * boundary included).  k = 0 maps to patch 0.  atan2 only picks where the
 * search starts. */
int32_t orc_project(const orc_model *m, double kx, double ky)
{
    kx = orc_fold(kx);
    ky = orc_fold(ky);
    if (kx == 0.0 && ky == 0.0) return 0;
    int N = m->N;
    double th = atan2(ky, kx);
    if (th < 0.0) th += TWO_PI_D;
    int j0 = (int)floor(th / m->dth);
    j0 = ((j0 % N) + N) % N;
    for (int d = 0; d <= N / 2; d++) {
        int ja = ((j0 + d) % N + N) % N;
        if (in_sector(m, ja, kx, ky)) return ja;
        int jb = ((j0 - d) % N + N) % N;
        if (in_sector(m, jb, kx, ky)) return jb;
    }
    return 0;
}

/* ------------------------------------------------------------------ G2/G3 build */
static void wedge_src(int N, int n_ang, int J, int sp, int *o, int *j, int *s)
{
    int w = N / 8;
    *o = J / w;
    int r = J % w;
    if ((*o & 1) == 0) { *j = r; *s = sp; }
    else { *j = w - 1 - r; *s = n_ang - 1 - sp; }
}

/* Raw fine point (s, m) of patch j built directly from its angles. */
static void raw_point(const orc_model *m, int j, int s, int mm, double *x, double *y, double *wt)
{
    double dth = m->dth;
    double th = (double)j * dth + ((double)s + 0.5) * (dth / (double)m->p.n_ang);
    double c = cos(th), sn = sin(th);
    double R = ray_extent(c, sn);
    double r = ((double)mm + 0.5) * R / (double)m->p.n_rad;
    *x = r * c;
    *y = r * sn;
    *wt = r * (R / (double)m->p.n_rad) * (dth / (double)m->p.n_ang) / (4.0 * PI_D * PI_D);
}

static void raw_centre(const orc_model *m, int j, double *x, double *y)
{
    double th = ((double)j + 0.5) * m->dth;
    double c = cos(th), sn = sin(th);
    double R = ray_extent(c, sn);
    double r = ray_root(&m->p, c, sn, R);
    *x = r * c;
    *y = r * sn;
}

/* fine point (wedge or direct patch j, index s) of the energy-angle grid */
static void egrid_point(const orc_model *m, int j, int s, double *x, double *y, double *wt)
{
    const double *q = m->eg_pts + 3 * ((size_t)j * m->nf + s);
    *x = q[0];
    *y = q[1];
    *wt = q[2];
}

static int build_geometry(orc_model *m)
{
    int N = m->N, nf = m->nf, na = m->p.n_ang, nr = m->p.n_rad;
    int sym = (N % 8 == 0);
    if (sym) {
        int w = N / 8;
        double *bw = malloc(sizeof(double) * 2 * (w + 1));
        for (int r = 0; r < w; r++) { bw[2 * r] = cos((double)r * m->dth); bw[2 * r + 1] = sin((double)r * m->dth); }
        bw[2 * w] = sqrt(0.5);
        bw[2 * w + 1] = sqrt(0.5);
        for (int i = 0; i < N; i++) {
            int o = i / w, r = i % w;
            int src = (o & 1) ? w - r : r;
            c4v(o, bw[2 * src], bw[2 * src + 1], &m->bnd[2 * i], &m->bnd[2 * i + 1]);
        }
        free(bw);
        double *cw = malloc(sizeof(double) * 2 * w);
        for (int j = 0; j < w; j++) raw_centre(m, j, &cw[2 * j], &cw[2 * j + 1]);
        for (int J = 0; J < N; J++) {
            int o, j, s;
            wedge_src(N, na, J, 0, &o, &j, &s);
            c4v(o, cw[2 * j], cw[2 * j + 1], &m->kc[2 * J], &m->kc[2 * J + 1]);
        }
        free(cw);
        for (int J = 0; J < N; J++)
            for (int sp = 0; sp < na; sp++)
                for (int mm = 0; mm < nr; mm++) {
                    int o, j, s;
                    wedge_src(N, na, J, sp, &o, &j, &s);
                    double x, y, wt;
                    /* the energy-angle list keeps its order in every octant, so that
                     * its zero-weight padding stays at the end of each patch */
                    if (m->egrid) egrid_point(m, j, sp, &x, &y, &wt);
                    else raw_point(m, j, s, mm, &x, &y, &wt);
                    int idx = J * nf + sp * nr + mm;
                    c4v(o, x, y, &m->px[idx], &m->py[idx]);
                    m->w[idx] = wt;
                }
    } else {
        for (int i = 0; i < N; i++) { m->bnd[2 * i] = cos((double)i * m->dth); m->bnd[2 * i + 1] = sin((double)i * m->dth); }
        for (int J = 0; J < N; J++) raw_centre(m, J, &m->kc[2 * J], &m->kc[2 * J + 1]);
        for (int J = 0; J < N; J++)
            for (int s = 0; s < na; s++)
                for (int mm = 0; mm < nr; mm++) {
                    int idx = J * nf + s * nr + mm;
                    if (m->egrid) egrid_point(m, J, s, &m->px[idx], &m->py[idx], &m->w[idx]);
                    else raw_point(m, J, s, mm, &m->px[idx], &m->py[idx], &m->w[idx]);
                }
    }
    m->bnd[2 * N] = m->bnd[0];
    m->bnd[2 * N + 1] = m->bnd[1];
    /* normalise the polar weights: sum over the whole grid in index order (the
     * energy-angle weights are used as the quadrature gives them) */
    if (!m->egrid) {
        double S = 0.0;
        for (int i = 0; i < N * nf; i++) S += m->w[i];
        for (int i = 0; i < N * nf; i++) m->w[i] = m->w[i] / S;
    }
    for (int i = 0; i < N * nf; i++) m->xi[i] = eps_k(&m->p, m->px[i], m->py[i]);
    /* transfers */
    int t = 0;
    for (int i = 0; i < N; i++)
        for (int j = i; j < N; j++) {
            m->qpp[2 * t] = orc_fold(m->kc[2 * i] + m->kc[2 * j]);
            m->qpp[2 * t + 1] = orc_fold(m->kc[2 * i + 1] + m->kc[2 * j + 1]);
            m->rpp[i * N + j] = t;
            m->rpp[j * N + i] = t;
            t++;
        }
    m->qph[0] = 0.0;
    m->qph[1] = 0.0;
    for (int x = 0; x < N; x++) m->rph[x * N + x] = 0;
    t = 1;
    for (int x = 0; x < N; x++)
        for (int y = 0; y < N; y++) {
            if (x == y) continue;
            m->qph[2 * t] = orc_fold(m->kc[2 * x] - m->kc[2 * y]);
            m->qph[2 * t + 1] = orc_fold(m->kc[2 * x + 1] - m->kc[2 * y + 1]);
            m->rph[x * N + y] = t;
            t++;
        }
    return 0;
}

orc_model *orc_create(const orc_params *p)
{
    if (!p) return NULL;
    if (p->N < 4 || p->N > 256 || p->N % 4 != 0) return NULL;
    if (p->n_rad < 1 || p->n_ang < 1 || p->n_rad * p->n_ang > 65536) return NULL;
    if (!isfinite(p->t) || !isfinite(p->tp) || !isfinite(p->mu) || !isfinite(p->U)) return NULL;
    orc_model *m = calloc(1, sizeof(orc_model));
    m->p = *p;
    m->N = p->N;
    m->nf = p->n_rad * p->n_ang;
    m->Tpp = p->N * (p->N + 1) / 2;
    m->Tph = p->N * (p->N - 1) + 1;
    m->dth = TWO_PI_D / (double)p->N;
    size_t np = (size_t)m->N * m->nf;
    m->kc = calloc(2 * m->N, sizeof(double));
    m->bnd = calloc(2 * (m->N + 1), sizeof(double));
    m->px = calloc(np, sizeof(double));
    m->py = calloc(np, sizeof(double));
    m->w = calloc(np, sizeof(double));
    m->xi = calloc(np, sizeof(double));
    m->qpp = calloc(2 * m->Tpp, sizeof(double));
    m->qph = calloc(2 * m->Tph, sizeof(double));
    m->rpp = calloc((size_t)m->N * m->N, sizeof(int32_t));
    m->rph = calloc((size_t)m->N * m->N, sizeof(int32_t));
    build_geometry(m);
    return m;
}

void orc_destroy(orc_model *m)
{
    if (!m) return;
    free(m->kc); free(m->bnd); free(m->px); free(m->py); free(m->w); free(m->xi);
    free(m->qpp); free(m->qph); free(m->rpp); free(m->rph); free(m->eg_pts);
    free(m);
}

/* ------------------------------------------------------------------ energy-angle grid */
/* The paper's quadrature (Sec. 4): the Brillouin-zone integral split into an
 * outer integral over energy, on a fixed grid of equidistant midpoints across
 * the band, and an inner integral along the line of that energy by a locally
 * adaptive midpoint rule (readings in the design notes).  The inner coordinate
 * is the angle theta of the ray from Gamma: eps increases monotonically along
 * every ray (|t'| < t/2), so energy E is met at one radius r(E, theta) or not
 * at all inside the zone, and d^2k = r dr dtheta = r / (d eps/dr) dE dtheta. */

/* density r / (d eps / dr) at the point of energy E on the ray (c, s), or 0 when
 * the ray does not reach E inside the zone; the point in *x, *y */
static double energy_density(const orc_params *p, double c, double s, double E, double *x, double *y)
{
    double R = ray_extent(c, s);
    *x = 0.0;
    *y = 0.0;
    if (!(eps_k(p, R * c, R * s) >= E)) return 0.0;
    double lo = 0.0, hi = R;
    for (int it = 0; it < 100; it++) {
        double mid = 0.5 * (lo + hi);
        if (eps_k(p, mid * c, mid * s) < E) lo = mid;
        else hi = mid;
    }
    double r = 0.5 * (lo + hi);
    double kx = r * c, ky = r * s;
    double sx = sin(kx), sy = sin(ky), cx = cos(kx), cy = cos(ky);
    double dx = (2.0 * p->t) * sx + (4.0 * p->tp) * (sx * cy);
    double dy = (2.0 * p->t) * sy + (4.0 * p->tp) * (cx * sy);
    double dedr = c * dx + s * dy;
    *x = kx;
    *y = ky;
    if (!(dedr > 0.0)) return 0.0;
    return r / dedr;
}

typedef struct {
    double *pts;          /* growing list of x, y, w */
    int n, cap;
} egrid_list;

static void eg_push(egrid_list *L, double x, double y, double w)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 256;
        L->pts = realloc(L->pts, sizeof(double) * 3 * L->cap);
    }
    L->pts[3 * L->n] = x;
    L->pts[3 * L->n + 1] = y;
    L->pts[3 * L->n + 2] = w;
    L->n++;
}

/* One cell [a, a + h) of the trisection midpoint rule on the shell of energy E
 * (weight factor dE / (2 pi)^2 in wf) whose midpoint density fmid is known.  The
 * three thirds' midpoints give I3; the cell's own midpoint gives I1 (it is the
 * middle third's midpoint, so refining reuses it).  A cell is refined while
 * |I3 - I1| exceeds its share of the shell's target, tol_rate * h (tol_rate =
 * rtol I_shell / 2 pi), and its thirds are above the deepest level; otherwise its
 * three thirds are the quadrature points (zero-density points dropped). */
static void eg_cell(const orc_params *p, double E, double wf, double a, double h, double fmid, double xm, double ym,
                    int level, int max_level, double tol_rate, egrid_list *L)
{
    double tol = tol_rate * h;
    double h3 = h / 3.0;
    double t1 = a + 0.5 * h3, t3 = a + 2.0 * h3 + 0.5 * h3;
    double x1, y1, x3, y3;
    double f1 = energy_density(p, cos(t1), sin(t1), E, &x1, &y1);
    double f3 = energy_density(p, cos(t3), sin(t3), E, &x3, &y3);
    double I1 = h * fmid;
    double I3 = h3 * (f1 + fmid + f3);
    if (level + 1 < max_level && fabs(I3 - I1) > tol) {
        eg_cell(p, E, wf, a, h3, f1, x1, y1, level + 1, max_level, tol_rate, L);
        eg_cell(p, E, wf, a + h3, h3, fmid, xm, ym, level + 1, max_level, tol_rate, L);
        eg_cell(p, E, wf, a + 2.0 * h3, h3, f3, x3, y3, level + 1, max_level, tol_rate, L);
        return;
    }
    if (f1 > 0.0) eg_push(L, x1, y1, wf * h3 * f1);
    if (fmid > 0.0) eg_push(L, xm, ym, wf * h3 * fmid);
    if (f3 > 0.0) eg_push(L, x3, y3, wf * h3 * f3);
}

/* Energy at the zone-boundary end of the ray at angle th: within each octant
 * (between consecutive multiples of pi/4) it is monotone in th, since on the
 * boundary edge it reads 2t + (4t' - 2t) cos(y) - mu with |y| rising to pi
 * towards the corner (|t'| < t/2). */
static double end_energy(const orc_params *p, double th)
{
    double c = cos(th), s = sin(th);
    double R = ray_extent(c, s);
    return eps_k(p, R * c, R * s);
}

/* The angles of [a0, a1) (inside one octant) whose ray reaches energy E: an
 * interval [*c0, *c1), empty when *c1 <= *c0.  The end energy is monotone, so
 * the covered part starts or ends at its one crossing of E (bisected). */
static void covered_piece(const orc_params *p, double E, double a0, double a1, double *c0, double *c1)
{
    double e0 = end_energy(p, a0), e1 = end_energy(p, a1);
    *c0 = a0;
    *c1 = a1;
    if (e0 >= E && e1 >= E) return;
    if (e0 < E && e1 < E) { *c1 = a0; return; }
    double lo = a0, hi = a1;
    int rising = (e1 >= E);
    for (int it = 0; it < 100; it++) {
        double mid = 0.5 * (lo + hi);
        if ((end_energy(p, mid) >= E) == rising) hi = mid;
        else lo = mid;
    }
    double x = 0.5 * (lo + hi);
    if (rising) *c0 = x;
    else *c1 = x;
}

/* The octant pieces of sector j: its angle range cut at multiples of pi/4;
 * returns their count (at most 3), bounds in cut[]. */
static int sector_pieces(const orc_model *m, int j, double *cut)
{
    double a = (double)j * m->dth, b = (double)(j + 1) * m->dth;
    int n = 0;
    cut[n++] = a;
    int k0 = (int)floor(a / (0.25 * PI_D)) + 1;
    for (int k = k0; (double)k * (0.25 * PI_D) < b; k++) cut[n++] = (double)k * (0.25 * PI_D);
    cut[n] = b;
    return n;
}

/* Points of sector j for every energy shell, shells in increasing energy, each
 * shell's points in increasing angle.  Only the covered part of each octant
 * piece is integrated (outside it the ray stays below E: no contour there), so
 * narrow contour arcs near the band top are never missed by the coarse samples.
 * I_shell[i]: a three-point-per-piece estimate of shell i's inner integral over
 * the whole circle, the scale of the relative target rtol. */
static void eg_sector(const orc_model *m, const orc_egrid *e, const double *I_shell, double Emin, double dE, int j,
                      egrid_list *L)
{
    double wf = dE / (4.0 * PI_D * PI_D);
    double cut[5];
    int np = sector_pieces(m, j, cut);
    for (int i = 0; i < e->n_E; i++) {
        double E = Emin + ((double)i + 0.5) * dE;
        for (int q = 0; q < np; q++) {
            double c0, c1;
            covered_piece(&m->p, E, cut[q], cut[q + 1], &c0, &c1);
            if (!(c1 > c0)) continue;
            double h = c1 - c0, tm = c0 + 0.5 * h, xm, ym;
            double fm = energy_density(&m->p, cos(tm), sin(tm), E, &xm, &ym);
            eg_cell(&m->p, E, wf, c0, h, fm, xm, ym, 0, e->max_level, e->rtol * I_shell[i] / TWO_PI_D, L);
        }
    }
}

/* three-point midpoint estimate of shell E's inner integral over sector j's covered pieces */
static double eg_coarse(const orc_model *m, double E, int j)
{
    double cut[5], acc = 0.0;
    int np = sector_pieces(m, j, cut);
    for (int q = 0; q < np; q++) {
        double c0, c1;
        covered_piece(&m->p, E, cut[q], cut[q + 1], &c0, &c1);
        if (!(c1 > c0)) continue;
        double h3 = (c1 - c0) / 3.0;
        for (int k = 0; k < 3; k++) {
            double t = c0 + ((double)k + 0.5) * h3, x, y;
            acc += h3 * energy_density(&m->p, cos(t), sin(t), E, &x, &y);
        }
    }
    return acc;
}

orc_model *orc_create_egrid(const orc_params *p, const orc_egrid *e)
{
    if (!p || !e) return NULL;
    if (p->N < 4 || p->N > 256 || p->N % 4 != 0) return NULL;
    if (e->n_E < 1 || e->max_level < 1 || e->max_level > 12 || !(e->rtol > 0.0)) return NULL;
    if (!isfinite(p->t) || !isfinite(p->tp) || !isfinite(p->mu) || !isfinite(p->U)) return NULL;
    if (!(fabs(p->tp) < 0.5 * fabs(p->t))) return NULL;   /* eps monotone along the rays */
    orc_model *m = calloc(1, sizeof(orc_model));
    m->p = *p;
    m->N = p->N;
    m->egrid = 1;
    m->dth = TWO_PI_D / (double)p->N;
    /* band edges: the minimum of eps at Gamma, the maximum at (pi, pi) */
    double Emin = eps_k(p, 0.0, 0.0), Emax = eps_k(p, PI_D, PI_D);
    double dE = (Emax - Emin) / (double)e->n_E;
    int sym = (m->N % 8 == 0);
    int nb = sym ? m->N / 8 : m->N;   /* sectors built: the first octant's, else all */
    /* the scale of each shell: three midpoints per sector of the sectors built */
    double *I_shell = calloc(e->n_E, sizeof(double));
    for (int i = 0; i < e->n_E; i++) {
        double E = Emin + ((double)i + 0.5) * dE, acc = 0.0;
        for (int j = 0; j < nb; j++) acc += eg_coarse(m, E, j);
        I_shell[i] = acc * (double)(m->N / nb);
    }
    egrid_list *lists = calloc(nb, sizeof(egrid_list));
    int nf = 1;
    for (int j = 0; j < nb; j++) {
        eg_sector(m, e, I_shell, Emin, dE, j, &lists[j]);
        if (lists[j].n > nf) nf = lists[j].n;
    }
    free(I_shell);
    /* every sector padded to nf points with zero weight at its first point */
    m->nf = nf;
    m->eg_pts = calloc((size_t)nb * nf * 3, sizeof(double));
    for (int j = 0; j < nb; j++) {
        for (int k = 0; k < nf; k++) {
            double *q = m->eg_pts + 3 * ((size_t)j * nf + k);
            if (k < lists[j].n) {
                q[0] = lists[j].pts[3 * k];
                q[1] = lists[j].pts[3 * k + 1];
                q[2] = lists[j].pts[3 * k + 2];
            } else {
                q[0] = lists[j].n ? lists[j].pts[0] : 0.0;
                q[1] = lists[j].n ? lists[j].pts[1] : 0.0;
                q[2] = 0.0;
            }
        }
        free(lists[j].pts);
    }
    free(lists);
    m->p.n_rad = 1;
    m->p.n_ang = nf;
    m->Tpp = m->N * (m->N + 1) / 2;
    m->Tph = m->N * (m->N - 1) + 1;
    size_t np = (size_t)m->N * m->nf;
    m->kc = calloc(2 * m->N, sizeof(double));
    m->bnd = calloc(2 * (m->N + 1), sizeof(double));
    m->px = calloc(np, sizeof(double));
    m->py = calloc(np, sizeof(double));
    m->w = calloc(np, sizeof(double));
    m->xi = calloc(np, sizeof(double));
    m->qpp = calloc(2 * m->Tpp, sizeof(double));
    m->qph = calloc(2 * m->Tph, sizeof(double));
    m->rpp = calloc((size_t)m->N * m->N, sizeof(int32_t));
    m->rph = calloc((size_t)m->N * m->N, sizeof(int32_t));
    build_geometry(m);
    return m;
}

int32_t orc_N(const orc_model *m) { return m->N; }
int32_t orc_nf(const orc_model *m) { return m->nf; }
int32_t orc_num_pp(const orc_model *m) { return m->Tpp; }
int32_t orc_num_ph(const orc_model *m) { return m->Tph; }
int32_t orc_row_pp(const orc_model *m, int32_t j1, int32_t j2) { return m->rpp[j1 * m->N + j2]; }
int32_t orc_row_ph(const orc_model *m, int32_t x, int32_t y) { return m->rph[x * m->N + y]; }

void orc_tables(const orc_model *m, double *kc, double *bnd, double *fine,
                double *qpp, double *qph, int32_t *idx4)
{
    int N = m->N;
    if (kc) memcpy(kc, m->kc, sizeof(double) * 2 * N);
    if (bnd) memcpy(bnd, m->bnd, sizeof(double) * 2 * (N + 1));
    if (fine)
        for (int i = 0; i < N * m->nf; i++) {
            fine[4 * i] = m->px[i];
            fine[4 * i + 1] = m->py[i];
            fine[4 * i + 2] = m->w[i];
            fine[4 * i + 3] = m->xi[i];
        }
    if (qpp) memcpy(qpp, m->qpp, sizeof(double) * 2 * m->Tpp);
    if (qph) memcpy(qph, m->qph, sizeof(double) * 2 * m->Tph);
    if (idx4)
        for (int a = 0; a < N; a++)
            for (int b = 0; b < N; b++)
                for (int c = 0; c < N; c++) {
                    double x = (m->kc[2 * a] + m->kc[2 * b]) - m->kc[2 * c];
                    double y = (m->kc[2 * a + 1] + m->kc[2 * b + 1]) - m->kc[2 * c + 1];
                    idx4[(a * N + b) * N + c] = orc_project(m, orc_fold(x), orc_fold(y));
                }
}

/* ------------------------------------------------------------------ G4 */
/* sech^2 x and tanh x from e = exp(-2|x|): no overflow for large |x|. */
static void sech2_tanh(double x, double *S, double *tau)
{
    double e = exp(-2.0 * fabs(x));
    double d = 1.0 + e;
    *S = 4.0 * e / (d * d);
    double th = (1.0 - e) / d;
    *tau = (x < 0.0) ? -th : th;
}

#define ORC_DELTA 2e-3

/* Divided difference of h(x) = x sech^2 x; Taylor branch
 * h'(m) + d^2 h'''(m)/24 for |d| < delta, m = (x+y)/2, with
 * h' = S(1 - 2 x tau), h''' = 12S - 18S^2 - 8 x S tau (1 - 3S). */
static double div_h(double x, double y)
{
    double d = x - y;
    if (fabs(d) < ORC_DELTA) {
        double mid = 0.5 * (x + y), S, tau;
        sech2_tanh(mid, &S, &tau);
        double h1 = S * (1.0 - 2.0 * mid * tau);
        double h3 = 12.0 * S - 18.0 * S * S - 8.0 * mid * S * tau * (1.0 - 3.0 * S);
        return h1 + d * d * h3 / 24.0;
    }
    double Sx, tx, Sy, ty;
    sech2_tanh(x, &Sx, &tx);
    sech2_tanh(y, &Sy, &ty);
    return (x * Sx - y * Sy) / d;
}

/* Divided difference of tanh; Taylor branch S(m) + d^2 (4S - 6S^2)(m)/24. */
static double div_tanh(double x, double y)
{
    double d = x - y;
    if (fabs(d) < ORC_DELTA) {
        double mid = 0.5 * (x + y), S, tau;
        sech2_tanh(mid, &S, &tau);
        return S + d * d * (4.0 * S - 6.0 * S * S) / 24.0;
    }
    double Sx, tx, Sy, ty;
    sech2_tanh(x, &Sx, &tx);
    sech2_tanh(y, &Sy, &ty);
    return (tx - ty) / d;
}

/* Static bubbles at zero external frequency, a = xi1/2T, b = xi2/2T:
 *   L_ph = (f(xi1)-f(xi2))/(xi2-xi1) = D[tanh](a, b)/(4T)
 *   L_pp = (1-f(xi1)-f(xi2))/(xi1+xi2) = D[tanh](a,-b)/(4T)
 *   dL_ph/dT = -D[h](a, b)/(4T^2),  dL_pp/dT = -D[h](a,-b)/(4T^2). */
double orc_L(int32_t kind, int32_t deriv, double xi1, double xi2, double T)
{
    double a = xi1 / (2.0 * T);
    double b = xi2 / (2.0 * T);
    if (kind == 1) b = -b;
    if (deriv) return -div_h(a, b) / (4.0 * T * T);
    return div_tanh(a, b) / (4.0 * T);
}

/* ------------------------------------------------------------------ G5 */
/* second loop line of fine point i for transfer row t: q - p (pp) or p + Q (ph) */
static void second_line(const orc_model *m, int kind, int t, int i, double *kx, double *ky)
{
    if (kind == 1) {
        *kx = orc_fold(m->qpp[2 * t] - m->px[i]);
        *ky = orc_fold(m->qpp[2 * t + 1] - m->py[i]);
    } else {
        *kx = orc_fold(m->px[i] + m->qph[2 * t]);
        *ky = orc_fold(m->py[i] + m->qph[2 * t + 1]);
    }
}

void orc_bins(const orc_model *m, int32_t kind, int32_t *out)
{
    int T = kind == 1 ? m->Tpp : m->Tph;
    int np = m->N * m->nf;
#pragma omp parallel for schedule(dynamic, 4) num_threads(NT)
    for (int t = 0; t < T; t++)
        for (int i = 0; i < np; i++) {
            double kx, ky;
            second_line(m, kind, t, i, &kx, &ky);
            out[(size_t)t * np + i] = orc_project(m, kx, ky);
        }
}

/* B_t(a,b) = sum over fine points p in patch a whose second line lies in
 * patch b of w_p L(xi_p, eps(second line)); with a self-energy S (one value
 * per patch, nullable) each line's energy carries its own patch's S:
 * L(xi_p + S_a, eps(second line) + S_b). */
static void bubble_kind(const orc_model *m, int kind, double T, int deriv, const double *S, double *B)
{
    int N = m->N, nf = m->nf;
    int Tn = kind == 1 ? m->Tpp : m->Tph;
    size_t NN = (size_t)N * N;
#pragma omp parallel for schedule(dynamic, 2) num_threads(NT)
    for (int t = 0; t < Tn; t++) {
        double *Bt = B + (size_t)t * NN;
        memset(Bt, 0, sizeof(double) * NN);
        for (int a = 0; a < N; a++)
            for (int k = 0; k < nf; k++) {
                int i = a * nf + k;
                double kx, ky;
                second_line(m, kind, t, i, &kx, &ky);
                int b = orc_project(m, kx, ky);
                double xi1 = m->xi[i], xi2 = eps_k(&m->p, kx, ky);
                if (S) {
                    xi1 = xi1 + S[a];
                    xi2 = xi2 + S[b];
                }
                Bt[a * N + b] += m->w[i] * orc_L(kind, deriv, xi1, xi2, T);
            }
    }
}

void orc_bubbles(const orc_model *m, double T, int32_t deriv, double *Bpp, double *Bph)
{
    if (Bpp) bubble_kind(m, 1, T, deriv, NULL, Bpp);
    if (Bph) bubble_kind(m, 0, T, deriv, NULL, Bph);
}

void orc_bubbles_se(const orc_model *m, double T, int32_t deriv, const double *S, double *Bpp, double *Bph)
{
    if (Bpp) bubble_kind(m, 1, T, deriv, S, Bpp);
    if (Bph) bubble_kind(m, 0, T, deriv, S, Bph);
}

/* ------------------------------------------------------------------ G8 */
/* F(j1,j2,j3) = - sum_ab Bpp_q(a,b)  V(j1,j2,a) V(a,b,j3)            q  = k1+k2
 *               + sum_ab Bph_Qc(a,b) V(j1,a,b)  V(b,j2,j3)            Qc = k3-k2
 *               + sum_ab Bph_Qd(a,b) [ -2 V(j1,b,j3) V(a,j2,b)
 *                                      +  V(j1,b,a)  V(a,j2,b)
 *                                      +  V(j1,b,j3) V(j2,a,b) ]     Qd = k3-k1 */
#define VI(j1, j2, j3) V[((size_t)(j1) * N + (j2)) * N + (j3)]

void orc_contract(const orc_model *m, const double *Bpp, const double *Bph,
                  const double *V, double *F)
{
    int N = m->N;
    size_t NN = (size_t)N * N;
#pragma omp parallel for collapse(2) schedule(dynamic, 1) num_threads(NT)
    for (int j1 = 0; j1 < N; j1++)
        for (int j2 = 0; j2 < N; j2++)
            for (int j3 = 0; j3 < N; j3++) {
                const double *Bq = Bpp + (size_t)m->rpp[j1 * N + j2] * NN;
                const double *Bc = Bph + (size_t)m->rph[j3 * N + j2] * NN;
                const double *Bd = Bph + (size_t)m->rph[j3 * N + j1] * NN;
                double s = 0.0;
                for (int a = 0; a < N; a++)
                    for (int b = 0; b < N; b++)
                        s -= Bq[a * N + b] * VI(j1, j2, a) * VI(a, b, j3);
                for (int a = 0; a < N; a++)
                    for (int b = 0; b < N; b++)
                        s += Bc[a * N + b] * VI(j1, a, b) * VI(b, j2, j3);
                for (int a = 0; a < N; a++)
                    for (int b = 0; b < N; b++)
                        s += Bd[a * N + b] * (-2.0 * VI(j1, b, j3) * VI(a, j2, b)
                                              + VI(j1, b, a) * VI(a, j2, b)
                                              + VI(j1, b, j3) * VI(j2, a, b));
                F[((size_t)j1 * N + j2) * N + j3] = s;
            }
}

void orc_rhs(const orc_model *m, double T, const double *V, double *F)
{
    size_t NN = (size_t)m->N * m->N;
    double *Bpp = malloc(sizeof(double) * NN * m->Tpp);
    double *Bph = malloc(sizeof(double) * NN * m->Tph);
    orc_bubbles(m, T, 1, Bpp, Bph);
    orc_contract(m, Bpp, Bph, V, F);
    free(Bpp);
    free(Bph);
}

/* Brute force: the same three diagrams as a direct sum over every fine point,
 * projecting each second line on the spot, without bubble tensors. */
static double rhs_entry(const orc_model *m, double T, const double *V, const double *S, int j1, int j2, int j3)
{
    int N = m->N, nf = m->nf;
    const double *kc = m->kc;
    double qx = orc_fold(kc[2 * j1] + kc[2 * j2]), qy = orc_fold(kc[2 * j1 + 1] + kc[2 * j2 + 1]);
    double cx = orc_fold(kc[2 * j3] - kc[2 * j2]), cy = orc_fold(kc[2 * j3 + 1] - kc[2 * j2 + 1]);
    double dx = orc_fold(kc[2 * j3] - kc[2 * j1]), dy = orc_fold(kc[2 * j3 + 1] - kc[2 * j1 + 1]);
    double s = 0.0;
    for (int a = 0; a < N; a++)
        for (int k = 0; k < nf; k++) {
            int i = a * nf + k;
            double px = m->px[i], py = m->py[i], w = m->w[i], x1 = m->xi[i] + (S ? S[a] : 0.0);
            double kx, ky, v;
            int b;
            kx = orc_fold(qx - px); ky = orc_fold(qy - py);
            b = orc_project(m, kx, ky);
            v = w * orc_L(1, 1, x1, eps_k(&m->p, kx, ky) + (S ? S[b] : 0.0), T);
            s -= v * VI(j1, j2, a) * VI(a, b, j3);
            kx = orc_fold(px + cx); ky = orc_fold(py + cy);
            b = orc_project(m, kx, ky);
            v = w * orc_L(0, 1, x1, eps_k(&m->p, kx, ky) + (S ? S[b] : 0.0), T);
            s += v * VI(j1, a, b) * VI(b, j2, j3);
            kx = orc_fold(px + dx); ky = orc_fold(py + dy);
            b = orc_project(m, kx, ky);
            v = w * orc_L(0, 1, x1, eps_k(&m->p, kx, ky) + (S ? S[b] : 0.0), T);
            s += v * (-2.0 * VI(j1, b, j3) * VI(a, j2, b) + VI(j1, b, a) * VI(a, j2, b)
                      + VI(j1, b, j3) * VI(j2, a, b));
        }
    return s;
}

void orc_rhs_entries(const orc_model *m, double T, const double *V, int64_t n,
                     const int32_t *j123, double *out)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(NT)
    for (int64_t e = 0; e < n; e++)
        out[e] = rhs_entry(m, T, V, NULL, j123[3 * e], j123[3 * e + 1], j123[3 * e + 2]);
}

void orc_rhs_entries_se(const orc_model *m, double T, const double *V, const double *S, int64_t n,
                        const int32_t *j123, double *out)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(NT)
    for (int64_t e = 0; e < n; e++)
        out[e] = rhs_entry(m, T, V, S, j123[3 * e], j123[3 * e + 1], j123[3 * e + 2]);
}

/* ------------------------------------------------------------------ self-energy */
/* The self-energy extension the paper names (Sec. 2) in its simplest form (a
 * reading): a static self-energy S_j, one value per patch, flowing with the
 * vertex.  Every loop line carries its patch's S (bubble_kind), and S flows by
 * the one-loop tadpole with the flowing vertex and the temperature derivative
 * of the occupation at fixed S:
 *   dS_j/dT = sum_a D_a [2 V(j, a, j) - V(a, j, j)],
 *   D_a = sum_{p in a} w_p d/dT n_F((xi_p + S_a)/T),
 *   d/dT n_F(x/T) = x/(4 T^2) sech^2(x/2T)   (x fixed).
 * The bracket is the spin sum of the antisymmetrised vertex at k3 = k1 (direct
 * term 2V, exchange term V with the legs crossed); at first order with V = U
 * it is the Hartree-Fock shift U n per spin. */
void orc_dsigma(const orc_model *m, double T, const double *V, const double *S, double *dS)
{
    int N = m->N, nf = m->nf;
    double *D = malloc(sizeof(double) * N);
    for (int a = 0; a < N; a++) {
        double acc = 0.0;
        for (int k = 0; k < nf; k++) {
            int i = a * nf + k;
            double x = m->xi[i] + (S ? S[a] : 0.0);
            double Sh, tau;
            sech2_tanh(x / (2.0 * T), &Sh, &tau);
            acc += m->w[i] * (x / (4.0 * T * T) * Sh);
        }
        D[a] = acc;
    }
    for (int j = 0; j < N; j++) {
        double acc = 0.0;
        for (int a = 0; a < N; a++) acc += D[a] * (2.0 * VI(j, a, j) - VI(a, j, j));
        dS[j] = acc;
    }
    free(D);
}

void orc_rhs_se(const orc_model *m, double T, const double *V, const double *S, double *F, double *dS)
{
    size_t NN = (size_t)m->N * m->N;
    double *Bpp = malloc(sizeof(double) * NN * m->Tpp);
    double *Bph = malloc(sizeof(double) * NN * m->Tph);
    orc_bubbles_se(m, T, 1, S, Bpp, Bph);
    orc_contract(m, Bpp, Bph, V, F);
    free(Bpp);
    free(Bph);
    orc_dsigma(m, T, V, S, dS);
}

/* ------------------------------------------------------------------ steppers */
static double maxabs(const double *y, int64_t n)
{
    double mx = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double a = fabs(y[i]);
        if (!(a <= mx)) mx = a;   /* propagates NaN */
    }
    return mx;
}

static int all_finite(const double *y, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(y[i])) return 0;
    return 1;
}

/* classical fourth-order Runge-Kutta, uniform steps s_i = s0 + i h */
int32_t orc_rk4(orc_ode_fn f, void *ctx, int64_t n, double *y, double s0, double s1,
                int32_t nsteps, double vmax, orc_ode_result *r)
{
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *yt = malloc(sizeof(double) * n);
    double h = (s1 - s0) / (double)nsteps;
    orc_ode_result res = {ORC_STOP_TMIN, s1, NAN, NAN, 0, 0, 0, 4};
    double m_prev = maxabs(y, n);
    for (int st = 0; st < nsteps; st++) {
        double s = s0 + (double)st * h;
        f(ctx, s, y, k1, n);
        for (int64_t i = 0; i < n; i++) yt[i] = y[i] + 0.5 * h * k1[i];
        f(ctx, s + 0.5 * h, yt, k2, n);
        for (int64_t i = 0; i < n; i++) yt[i] = y[i] + 0.5 * h * k2[i];
        f(ctx, s + 0.5 * h, yt, k3, n);
        for (int64_t i = 0; i < n; i++) yt[i] = y[i] + h * k3[i];
        f(ctx, s + h, yt, k4, n);
        for (int64_t i = 0; i < n; i++)
            y[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        res.rhs_evals += 4;
        res.accepted++;
        if (!all_finite(y, n)) { res.reason = ORC_STOP_NONFINITE; res.s_end = s + h; break; }
        double mx = maxabs(y, n);
        if (mx > vmax) {
            res.reason = ORC_STOP_DIVERGED;
            res.s_end = res.s_c = s + h;
            res.s_c_interp = s + (vmax - m_prev) / (mx - m_prev) * h;
            break;
        }
        m_prev = mx;
    }
    free(k1); free(k2); free(k3); free(k4); free(yt);
    if (r) *r = res;
    return res.reason;
}

/* Dormand & Prince (1980) 5(4) coefficients */
static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0},
    {1.0 / 5},
    {3.0 / 40, 9.0 / 40},
    {44.0 / 45, -56.0 / 15, 32.0 / 9},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double DP_B5[7] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192,
                                -2187.0 / 6784, 11.0 / 84, 0.0};
static const double DP_B4[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

/* G10: err = max_i |y5-y4| / (atol + rtol max(|y|,|y5|)); accept if err <= 1;
 * h <- h clamp(0.9 err^-1/5, 0.2, 5); last step clipped onto s_min; stop after
 * an accepted step when max|y| > vmax or s reached s_min. */
int32_t orc_dp54(orc_ode_fn f, void *ctx, int64_t n, double *y, double s0, double s_min,
                 double h0, double rtol, double atol, double vmax, int32_t max_steps,
                 orc_ode_result *r, double *logbuf, int32_t log_cap)
{
    double *k[7];
    for (int i = 0; i < 7; i++) k[i] = malloc(sizeof(double) * n);
    double *yt = malloc(sizeof(double) * n), *y5 = malloc(sizeof(double) * n);
    orc_ode_result res = {ORC_STOP_NONE, s0, NAN, NAN, 0, 0, 0, 0};
    double s = s0, h = h0;
    double dir = (s_min < s0) ? -1.0 : 1.0;     /* integrate towards s_min */
    if (h * dir < 0.0) h = -h;
    double m_prev = maxabs(y, n), s_prev = s;
    f(ctx, s, y, k[0], n);
    res.rhs_evals = 1;
    for (;;) {
        if (max_steps > 0 && res.accepted >= max_steps) { res.reason = ORC_STOP_MAXSTEPS; break; }
        if (!(fabs(h) > 1e-14 * (1.0 + fabs(s)))) { res.reason = ORC_STOP_HMIN; break; }
        int last = 0;
        if ((s + h - s_min) * dir >= 0.0) { h = s_min - s; last = 1; }
        for (int st = 1; st < 7; st++) {
            for (int64_t i = 0; i < n; i++) {
                double acc = 0.0;
                for (int j = 0; j < st; j++) acc += DP_A[st][j] * k[j][i];
                yt[i] = y[i] + h * acc;
            }
            if (st == 6) memcpy(y5, yt, sizeof(double) * n);
            f(ctx, s + DP_C[st] * h, yt, k[st], n);
            res.rhs_evals++;
        }
        double err = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double e = 0.0;
            for (int j = 0; j < 7; j++) e += (DP_B5[j] - DP_B4[j]) * k[j][i];
            e = fabs(h * e);
            double sc = atol + rtol * fmax(fabs(y[i]), fabs(y5[i]));
            double q = e / sc;
            if (!(q <= err)) err = q;
        }
        if (!isfinite(err) || !all_finite(y5, n)) { res.reason = ORC_STOP_NONFINITE; break; }
        double fac = err == 0.0 ? 5.0 : 0.9 * pow(err, -0.2);
        if (fac < 0.2) fac = 0.2;
        if (fac > 5.0) fac = 5.0;
        if (err <= 1.0) {
            memcpy(y, y5, sizeof(double) * n);
            double *swap = k[0]; k[0] = k[6]; k[6] = swap;   /* FSAL */
            double s_new = last ? s_min : s + h;
            res.accepted++;
            if (res.accepted == 1) res.first_step_rhs = res.rhs_evals;
            double mx = maxabs(y, n);
            if (logbuf && res.accepted <= log_cap) {
                double *L = logbuf + 6 * (res.accepted - 1);
                L[0] = s_new; L[1] = h; L[2] = err; L[3] = mx; L[4] = res.rhs_evals; L[5] = res.rejected;
            }
            s_prev = s;
            s = s_new;
            if (mx > vmax) {
                res.reason = ORC_STOP_DIVERGED;
                res.s_c = s;
                res.s_c_interp = s_prev + (vmax - m_prev) / (mx - m_prev) * (s - s_prev);
                break;
            }
            m_prev = mx;
            if (last) { res.reason = ORC_STOP_TMIN; break; }
            h = h * fac;
        } else {
            res.rejected++;
            h = h * fac;
        }
    }
    res.s_end = s;
    for (int i = 0; i < 7; i++) free(k[i]);
    free(yt); free(y5);
    if (r) *r = res;
    return res.reason;
}

/* ------------------------------------------------------------------ G9 flow */
typedef struct { const orc_model *m; } flow_ctx;

/* dV/ds = T F(V, T) with T = exp(s) */
static void flow_rhs(void *ctx, double s, const double *y, double *dy, int64_t n)
{
    const orc_model *m = ((flow_ctx *)ctx)->m;
    double T = exp(s);
    orc_rhs(m, T, y, dy);
    for (int64_t i = 0; i < n; i++) dy[i] = T * dy[i];
}

int32_t orc_flow(const orc_model *m, const orc_flow_opts *o, double *V, orc_ode_result *r,
                 double *logbuf, int32_t log_cap)
{
    flow_ctx c = {m};
    int64_t n = (int64_t)m->N * m->N * m->N;
    double s0 = log(o->T0), s1 = log(o->T_min);
    if (o->stepper == 0)
        return orc_rk4(flow_rhs, &c, n, V, s0, s1, o->fixed_steps, o->vmax, r);
    return orc_dp54(flow_rhs, &c, n, V, s0, s1, o->h0, o->rtol, o->atol, o->vmax,
                    o->max_steps, r, logbuf, log_cap);
}

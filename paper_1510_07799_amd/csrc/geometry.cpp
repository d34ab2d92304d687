// Host geometry of the N-patch discretisation (built once per context).
//
// Sec. 4 of the paper discretises the vertex on N momentum patches and
// integrates each one-loop diagram over the 2D Brillouin zone; it does not
// define the patches.  The construction used here (and, written separately,
// by the CPU oracle, so that every integer map agrees bit for bit):
//   - patch j = angular sector [j, j+1) * 2pi/N around Gamma, centre on the
//     Fermi surface along the sector's mid ray (first sign change of eps over
//     1024 nodes on (0, R], bisected 100 times; else the node of least |eps|);
//   - n_ang sub-rays at (s + 1/2) dth/n_ang, n_rad midpoints r_m = (m+1/2) R/n_rad,
//     weight r dr dtheta / (2pi)^2 normalised to a unit sum;
//   - for N % 8 == 0 everything is computed on the octant [0, pi/4] and
//     mapped to the other seven by exact swaps / sign flips, so the grid is
//     bitwise C4v symmetric.
// Every expression below is evaluated in the written order with no FP
// contraction (compiled with -ffp-contract=off); the libm calls are the host's.
#include <cmath>

#include "frg_internal.h"

namespace frg {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;

struct Disp {
    double mt2, mt4p, mu;  // -2t, 4t', mu
    double operator()(double kx, double ky) const {
        const double cx = std::cos(kx), cy = std::cos(ky);
        return mt2 * (cx + cy) - mt4p * (cx * cy) - mu;
    }
};

// exact point-group action: element o of C4v on (x, y)
inline void apply_c4v(int o, double x, double y, double &ox, double &oy) {
    const double X[8] = {x, y, -y, -x, -x, -y, y, x};
    const double Y[8] = {y, x, x, y, -y, -x, -x, -y};
    ox = X[o];
    oy = Y[o];
}

inline double zone_extent(double c, double s) {
    return kPi / std::fmax(std::fabs(c), std::fabs(s));
}

double fermi_radius(const Disp &eps, double c, double s, double R) {
    double r0 = R * 1.0 / 1024.0;
    double e0 = eps(r0 * c, r0 * s);
    double rbest = r0, ebest = std::fabs(e0);
    for (int i = 2; i <= 1024; ++i) {
        const double r1 = R * static_cast<double>(i) / 1024.0;
        const double e1 = eps(r1 * c, r1 * s);
        const bool p0 = e0 >= 0.0, p1 = e1 >= 0.0;
        if (p0 != p1) {
            double lo = r0, hi = r1;
            for (int it = 0; it < 100; ++it) {
                const double mid = 0.5 * (lo + hi);
                if ((eps(mid * c, mid * s) >= 0.0) == p0) lo = mid; else hi = mid;
            }
            return 0.5 * (lo + hi);
        }
        if (std::fabs(e1) < ebest) { ebest = std::fabs(e1); rbest = r1; }
        r0 = r1;
        e0 = e1;
    }
    return rbest;
}

struct RawPoint { double x, y, w; };

RawPoint sector_point(const Geometry &g, int j, int s, int m) {
    const double th = static_cast<double>(j) * g.dth +
                      (static_cast<double>(s) + 0.5) * (g.dth / static_cast<double>(g.n_ang));
    const double c = std::cos(th), sn = std::sin(th);
    const double R = zone_extent(c, sn);
    const double r = (static_cast<double>(m) + 0.5) * R / static_cast<double>(g.n_rad);
    RawPoint p;
    p.x = r * c;
    p.y = r * sn;
    p.w = r * (R / static_cast<double>(g.n_rad)) * (g.dth / static_cast<double>(g.n_ang)) /
          (4.0 * kPi * kPi);
    return p;
}

void sector_centre(const Geometry &g, const Disp &eps, int j, double &x, double &y) {
    const double th = (static_cast<double>(j) + 0.5) * g.dth;
    const double c = std::cos(th), sn = std::sin(th);
    const double r = fermi_radius(eps, c, sn, zone_extent(c, sn));
    x = r * c;
    y = r * sn;
}

}  // namespace

double fold_bz(double x) {
    while (x >= kPi) x -= kTwoPi;
    while (x < -kPi) x += kTwoPi;
    return x;
}

// sector test with the products rounded separately (no fused multiply-add)
static inline bool host_in_sector(const double *b0, const double *b1, double kx, double ky) {
    const double u0 = b0[0] * ky, v0 = b0[1] * kx;
    const double u1 = b1[0] * ky, v1 = b1[1] * kx;
    return (u0 - v0) >= 0.0 && (u1 - v1) < 0.0;
}

int32_t host_patch(const Geometry &g, double kx, double ky) {
    kx = fold_bz(kx);
    ky = fold_bz(ky);
    if (kx == 0.0 && ky == 0.0) return 0;
    double th = std::atan2(ky, kx);
    if (th < 0.0) th += kTwoPi;
    const int N = g.N;
    int j0 = static_cast<int>(std::floor(th / g.dth)) % N;
    if (j0 < 0) j0 += N;
    for (int d = 0; d <= N / 2; ++d) {
        for (int sgn = 0; sgn < 2; ++sgn) {
            int j = sgn ? j0 - d : j0 + d;
            j = ((j % N) + N) % N;
            if (host_in_sector(&g.bnd[2 * j], &g.bnd[2 * (j + 1)], kx, ky)) return j;
        }
    }
    return 0;
}

void host_idx4(const Geometry &g, int32_t *out) {
    const int N = g.N;
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            for (int c = 0; c < N; ++c) {
                const double x = (g.kc[2 * a] + g.kc[2 * b]) - g.kc[2 * c];
                const double y = (g.kc[2 * a + 1] + g.kc[2 * b + 1]) - g.kc[2 * c + 1];
                out[(static_cast<size_t>(a) * N + b) * N + c] = host_patch(g, fold_bz(x), fold_bz(y));
            }
}

void build_transfers(Geometry &g);

void build_geometry(const frg_params &p, Geometry &g) {
    g.N = p.N;
    g.n_rad = p.n_rad;
    g.n_ang = p.n_ang;
    g.nf = p.n_rad * p.n_ang;
    g.np = g.N * g.nf;
    g.Tpp = g.N * (g.N + 1) / 2;
    g.Tph = g.N * (g.N - 1) + 1;
    g.t = p.t; g.tp = p.tp; g.mu = p.mu; g.U = p.U;
    g.dth = kTwoPi / static_cast<double>(g.N);
    const Disp eps{-2.0 * p.t, 4.0 * p.tp, p.mu};
    const int N = g.N, nf = g.nf;
    g.kc.assign(2 * N, 0.0);
    g.bnd.assign(2 * (N + 1), 0.0);
    g.px.assign(g.np, 0.0);
    g.py.assign(g.np, 0.0);
    g.w.assign(g.np, 0.0);
    g.xi.assign(g.np, 0.0);

    if (N % 8 == 0) {
        const int q = N / 8;  // patches per octant
        // octant boundaries 0..q (q = the diagonal)
        std::vector<double> ob(2 * (q + 1));
        for (int r = 0; r < q; ++r) {
            ob[2 * r] = std::cos(static_cast<double>(r) * g.dth);
            ob[2 * r + 1] = std::sin(static_cast<double>(r) * g.dth);
        }
        ob[2 * q] = std::sqrt(0.5);
        ob[2 * q + 1] = std::sqrt(0.5);
        for (int i = 0; i < N; ++i) {
            const int o = i / q, r = i % q;
            const int src = (o & 1) ? q - r : r;
            apply_c4v(o, ob[2 * src], ob[2 * src + 1], g.bnd[2 * i], g.bnd[2 * i + 1]);
        }
        // octant image of patch J: element o, source patch j, sub-ray reversal
        auto source = [q](int J, int &o, int &j, bool &rev) {
            o = J / q;
            rev = (o & 1) != 0;
            j = rev ? q - 1 - (J % q) : J % q;
        };
        std::vector<double> oc(2 * q);
        for (int j = 0; j < q; ++j) sector_centre(g, eps, j, oc[2 * j], oc[2 * j + 1]);
        for (int J = 0; J < N; ++J) {
            int o, j;
            bool rev;
            source(J, o, j, rev);
            apply_c4v(o, oc[2 * j], oc[2 * j + 1], g.kc[2 * J], g.kc[2 * J + 1]);
            for (int s = 0; s < g.n_ang; ++s) {
                const int ss = rev ? g.n_ang - 1 - s : s;
                for (int m = 0; m < g.n_rad; ++m) {
                    const RawPoint rp = sector_point(g, j, ss, m);
                    const size_t idx = static_cast<size_t>(J) * nf + s * g.n_rad + m;
                    apply_c4v(o, rp.x, rp.y, g.px[idx], g.py[idx]);
                    g.w[idx] = rp.w;
                }
            }
        }
    } else {
        for (int i = 0; i < N; ++i) {
            g.bnd[2 * i] = std::cos(static_cast<double>(i) * g.dth);
            g.bnd[2 * i + 1] = std::sin(static_cast<double>(i) * g.dth);
        }
        for (int J = 0; J < N; ++J) {
            sector_centre(g, eps, J, g.kc[2 * J], g.kc[2 * J + 1]);
            for (int s = 0; s < g.n_ang; ++s)
                for (int m = 0; m < g.n_rad; ++m) {
                    const RawPoint rp = sector_point(g, J, s, m);
                    const size_t idx = static_cast<size_t>(J) * nf + s * g.n_rad + m;
                    g.px[idx] = rp.x;
                    g.py[idx] = rp.y;
                    g.w[idx] = rp.w;
                }
        }
    }
    g.bnd[2 * N] = g.bnd[0];
    g.bnd[2 * N + 1] = g.bnd[1];

    double wsum = 0.0;
    for (int i = 0; i < g.np; ++i) wsum += g.w[i];
    for (int i = 0; i < g.np; ++i) g.w[i] = g.w[i] / wsum;
    for (int i = 0; i < g.np; ++i) g.xi[i] = eps(g.px[i], g.py[i]);
    build_transfers(g);
}

namespace {

// transfer momenta of the pp rows (k_i + k_j, i <= j) and ph rows (k_x - k_y,
// x != y; row 0 is Q = 0) from the patch centres
void build_transfers_impl(Geometry &g) {
    const int N = g.N;
    g.qpp.assign(2 * g.Tpp, 0.0);
    g.qph.assign(2 * g.Tph, 0.0);
    g.row_pp.assign(N * N, 0);
    g.row_ph.assign(N * N, 0);
    int t = 0;
    for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j, ++t) {
            g.qpp[2 * t] = fold_bz(g.kc[2 * i] + g.kc[2 * j]);
            g.qpp[2 * t + 1] = fold_bz(g.kc[2 * i + 1] + g.kc[2 * j + 1]);
            g.row_pp[i * N + j] = g.row_pp[j * N + i] = t;
        }
    t = 1;
    for (int x = 0; x < N; ++x)
        for (int y = 0; y < N; ++y) {
            if (x == y) { g.row_ph[x * N + y] = 0; continue; }
            g.qph[2 * t] = fold_bz(g.kc[2 * x] - g.kc[2 * y]);
            g.qph[2 * t + 1] = fold_bz(g.kc[2 * x + 1] - g.kc[2 * y + 1]);
            g.row_ph[x * N + y] = t++;
        }
}

}  // namespace

void build_transfers(Geometry &g) { build_transfers_impl(g); }

// ----------------------------------------------------------------- energy-angle grid
// Sec. 4 integrates over the zone with an outer fixed midpoint grid in energy
// and an inner locally adaptive midpoint rule along each energy.  Here the inner
// coordinate is the angle th of the ray from Gamma: for |t'| < t/2 eps rises
// along every ray inside the zone, so energy E is crossed once at radius r(E, th)
// or not at all, and d^2k = r / (d eps / dr) dE dth.  The bubble is binned by the
// loop momentum's patch, so the inner rule runs per patch sector, on each octant
// piece of it (where the end energy of the ray is monotone) over the angles whose
// ray reaches E.  A cell is cut in thirds (its midpoint becomes the middle
// third's) while its one- and three-point values differ by more than
// rtol * I_E * h / 2pi (I_E: a three-point-per-piece estimate of the shell's
// whole inner integral), to at most 3^max_level points per piece and shell.
// Weights are dE h r / (d eps / dr) / (2pi)^2, not normalised.  The arithmetic
// is written in the same order as the oracle's (each product and sum rounded as
// written, libm calls of the host), so the points agree bit for bit.
namespace {

struct EgridBuilder {
    const Disp &eps;
    double t2, tp4;      // 2t, 4t'
    int max_level;
    std::vector<double> pts;   // x, y, w of the sector being built

    // r / (d eps / dr) at the crossing of energy E on the ray (c, s), 0 when the
    // ray stays below E inside the zone; the crossing point in (x, y)
    double density(double c, double s, double E, double &x, double &y) const {
        const double R = zone_extent(c, s);
        x = 0.0;
        y = 0.0;
        if (!(eps(R * c, R * s) >= E)) return 0.0;
        double lo = 0.0, hi = R;
        for (int it = 0; it < 100; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (eps(mid * c, mid * s) < E) lo = mid; else hi = mid;
        }
        const double r = 0.5 * (lo + hi);
        const double kx = r * c, ky = r * s;
        const double sx = std::sin(kx), sy = std::sin(ky), cx = std::cos(kx), cy = std::cos(ky);
        const double gx = t2 * sx + tp4 * (sx * cy);
        const double gy = t2 * sy + tp4 * (cx * sy);
        const double dr = c * gx + s * gy;
        x = kx;
        y = ky;
        if (!(dr > 0.0)) return 0.0;
        return r / dr;
    }

    double end_energy(double th) const {
        const double c = std::cos(th), s = std::sin(th);
        const double R = zone_extent(c, s);
        return eps(R * c, R * s);
    }

    // angles of [a0, a1) (one octant piece) whose ray reaches E: [c0, c1)
    void covered(double E, double a0, double a1, double &c0, double &c1) const {
        const double e0 = end_energy(a0), e1 = end_energy(a1);
        c0 = a0;
        c1 = a1;
        if (e0 >= E && e1 >= E) return;
        if (e0 < E && e1 < E) {
            c1 = a0;
            return;
        }
        const bool rising = e1 >= E;
        double lo = a0, hi = a1;
        for (int it = 0; it < 100; ++it) {
            const double mid = 0.5 * (lo + hi);
            if ((end_energy(mid) >= E) == rising) hi = mid; else lo = mid;
        }
        const double x = 0.5 * (lo + hi);
        if (rising) c0 = x; else c1 = x;
    }

    // sector [j dth, (j+1) dth) cut at the multiples of pi/4 inside it
    static int pieces(double dth, int j, double *cut) {
        const double a = static_cast<double>(j) * dth, b = static_cast<double>(j + 1) * dth;
        int n = 0;
        cut[n++] = a;
        for (int k = static_cast<int>(std::floor(a / (0.25 * kPi))) + 1; static_cast<double>(k) * (0.25 * kPi) < b; ++k)
            cut[n++] = static_cast<double>(k) * (0.25 * kPi);
        cut[n] = b;
        return n;
    }

    // depth-first over the cells of one covered piece: a cell is (a, h, level,
    // its midpoint's density and point); children pushed right to left so they
    // are taken left to right
    void piece(double E, double wf, double c0, double h0, double tol_rate) {
        struct Cell { double a, h, f, x, y; int level; };
        std::vector<Cell> stack;
        Cell root{c0, h0, 0.0, 0.0, 0.0, 0};
        const double tm = c0 + 0.5 * h0;
        root.f = density(std::cos(tm), std::sin(tm), E, root.x, root.y);
        stack.push_back(root);
        while (!stack.empty()) {
            const Cell cl = stack.back();
            stack.pop_back();
            const double h3 = cl.h / 3.0;
            const double t1 = cl.a + 0.5 * h3, t3 = cl.a + 2.0 * h3 + 0.5 * h3;
            double x1, y1, x3, y3;
            const double f1 = density(std::cos(t1), std::sin(t1), E, x1, y1);
            const double f3 = density(std::cos(t3), std::sin(t3), E, x3, y3);
            const double one = cl.h * cl.f;
            const double three = h3 * (f1 + cl.f + f3);
            if (cl.level + 1 < max_level && std::fabs(three - one) > tol_rate * cl.h) {
                stack.push_back(Cell{cl.a + 2.0 * h3, h3, f3, x3, y3, cl.level + 1});
                stack.push_back(Cell{cl.a + h3, h3, cl.f, cl.x, cl.y, cl.level + 1});
                stack.push_back(Cell{cl.a, h3, f1, x1, y1, cl.level + 1});
                continue;
            }
            const double q = wf * h3;
            if (f1 > 0.0) { pts.push_back(x1); pts.push_back(y1); pts.push_back(q * f1); }
            if (cl.f > 0.0) { pts.push_back(cl.x); pts.push_back(cl.y); pts.push_back(q * cl.f); }
            if (f3 > 0.0) { pts.push_back(x3); pts.push_back(y3); pts.push_back(q * f3); }
        }
    }

    // three-point estimate of shell E's inner integral over sector j's covered pieces
    double coarse(double dth, double E, int j) const {
        double cut[5], acc = 0.0;
        const int n = pieces(dth, j, cut);
        for (int q = 0; q < n; ++q) {
            double c0, c1;
            covered(E, cut[q], cut[q + 1], c0, c1);
            if (!(c1 > c0)) continue;
            const double h3 = (c1 - c0) / 3.0;
            for (int k = 0; k < 3; ++k) {
                const double th = c0 + (static_cast<double>(k) + 0.5) * h3;
                double x, y;
                acc += h3 * density(std::cos(th), std::sin(th), E, x, y);
            }
        }
        return acc;
    }
};

}  // namespace

bool build_geometry_egrid(const frg_params &p, const frg_egrid &e, int max_nf, Geometry &g) {
    g.N = p.N;
    g.t = p.t; g.tp = p.tp; g.mu = p.mu; g.U = p.U;
    g.Tpp = g.N * (g.N + 1) / 2;
    g.Tph = g.N * (g.N - 1) + 1;
    g.dth = kTwoPi / static_cast<double>(g.N);
    g.egrid = true;
    const Disp eps{-2.0 * p.t, 4.0 * p.tp, p.mu};
    const int N = g.N;
    const bool sym = N % 8 == 0;
    const int nb = sym ? N / 8 : N;   // sectors built
    const double Emin = eps(0.0, 0.0), Emax = eps(kPi, kPi);
    const double dE = (Emax - Emin) / static_cast<double>(e.n_E);
    EgridBuilder B{eps, 2.0 * p.t, 4.0 * p.tp, e.max_level, {}};
    std::vector<double> I(e.n_E);
    for (int i = 0; i < e.n_E; ++i) {
        const double E = Emin + (static_cast<double>(i) + 0.5) * dE;
        double acc = 0.0;
        for (int j = 0; j < nb; ++j) acc += B.coarse(g.dth, E, j);
        I[i] = acc * static_cast<double>(N / nb);
    }
    const double wf = dE / (4.0 * kPi * kPi);
    std::vector<std::vector<double>> sec(nb);
    int most = 1;
    for (int j = 0; j < nb; ++j) {
        B.pts.clear();
        double cut[5];
        const int n = EgridBuilder::pieces(g.dth, j, cut);
        for (int i = 0; i < e.n_E; ++i) {
            const double E = Emin + (static_cast<double>(i) + 0.5) * dE;
            for (int q = 0; q < n; ++q) {
                double c0, c1;
                B.covered(E, cut[q], cut[q + 1], c0, c1);
                if (!(c1 > c0)) continue;
                B.piece(E, wf, c0, c1 - c0, e.rtol * I[i] / kTwoPi);
            }
        }
        sec[j].swap(B.pts);
        most = std::max(most, static_cast<int>(sec[j].size() / 3));
        if (most > max_nf) return false;
    }
    g.nf = (most + kSegPoints - 1) / kSegPoints * kSegPoints;
    if (g.nf > max_nf) return false;
    g.n_rad = 1;
    g.n_ang = g.nf;
    g.np = N * g.nf;
    g.kc.assign(2 * N, 0.0);
    g.bnd.assign(2 * (N + 1), 0.0);
    g.px.assign(g.np, 0.0);
    g.py.assign(g.np, 0.0);
    g.w.assign(g.np, 0.0);
    g.xi.assign(g.np, 0.0);
    g.count.assign(N, 0);
    // patch J takes sector j's list through C4v element o (order kept, padding
    // last: copies of the first point with zero weight)
    auto fill = [&](int J, int o, int j) {
        const std::vector<double> &L = sec[j];
        const int n = static_cast<int>(L.size() / 3);
        g.count[J] = n;
        const double x0 = n ? L[0] : 0.0, y0 = n ? L[1] : 0.0;
        for (int k = 0; k < g.nf; ++k) {
            const size_t idx = static_cast<size_t>(J) * g.nf + k;
            const bool live = k < n;
            apply_c4v(o, live ? L[3 * k] : x0, live ? L[3 * k + 1] : y0, g.px[idx], g.py[idx]);
            g.w[idx] = live ? L[3 * k + 2] : 0.0;
        }
    };
    if (sym) {
        const int q = N / 8;
        std::vector<double> ob(2 * (q + 1));
        for (int r = 0; r < q; ++r) {
            ob[2 * r] = std::cos(static_cast<double>(r) * g.dth);
            ob[2 * r + 1] = std::sin(static_cast<double>(r) * g.dth);
        }
        ob[2 * q] = std::sqrt(0.5);
        ob[2 * q + 1] = std::sqrt(0.5);
        for (int i = 0; i < N; ++i) {
            const int o = i / q, r = i % q;
            const int src = (o & 1) ? q - r : r;
            apply_c4v(o, ob[2 * src], ob[2 * src + 1], g.bnd[2 * i], g.bnd[2 * i + 1]);
        }
        std::vector<double> oc(2 * q);
        for (int j = 0; j < q; ++j) sector_centre(g, eps, j, oc[2 * j], oc[2 * j + 1]);
        for (int J = 0; J < N; ++J) {
            const int o = J / q;
            const int j = (o & 1) ? q - 1 - (J % q) : J % q;
            apply_c4v(o, oc[2 * j], oc[2 * j + 1], g.kc[2 * J], g.kc[2 * J + 1]);
            fill(J, o, j);
        }
    } else {
        for (int i = 0; i < N; ++i) {
            g.bnd[2 * i] = std::cos(static_cast<double>(i) * g.dth);
            g.bnd[2 * i + 1] = std::sin(static_cast<double>(i) * g.dth);
        }
        for (int J = 0; J < N; ++J) {
            sector_centre(g, eps, J, g.kc[2 * J], g.kc[2 * J + 1]);
            fill(J, 0, J);
        }
    }
    g.bnd[2 * N] = g.bnd[0];
    g.bnd[2 * N + 1] = g.bnd[1];
    for (int i = 0; i < g.np; ++i) g.xi[i] = eps(g.px[i], g.py[i]);
    build_transfers(g);
    return true;
}

}  // namespace frg

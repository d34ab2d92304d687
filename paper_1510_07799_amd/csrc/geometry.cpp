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

}  // namespace frg

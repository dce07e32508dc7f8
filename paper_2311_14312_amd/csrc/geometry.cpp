// Host-side geometry of a scene: Gauss-Legendre rules, arc-length
// parametrisation of cubic Beziers (App. B), panels, nodes and chord
// segments with their arc-length scale (App. A), the Legendre interpolation
// matrix (Sec. 5.2) and the boundary colours at the nodes (Sec. 5.3).
#include "geometry.h"

#include <algorithm>
#include <cmath>

namespace dc {

// Roots and weights of the n-point Gauss-Legendre rule on [-1, 1], by
// Newton's method on P_n evaluated with the three-term recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846264338327950288;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        // recompute the derivative at the converged root for the weight
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

static void bezier(const double* c, double t, double& x, double& y) {
    const double s = 1.0 - t;
    const double b0 = s * s * s, b1 = 3.0 * t * s * s, b2 = 3.0 * t * t * s, b3 = t * t * t;
    x = b0 * c[0] + b1 * c[2] + b2 * c[4] + b3 * c[6];
    y = b0 * c[1] + b1 * c[3] + b2 * c[5] + b3 * c[7];
}

static double speed(const double* c, double t) {
    const double s = 1.0 - t;
    const double a = 3.0 * s * s, b = 6.0 * t * s, d = 3.0 * t * t;
    const double dx = a * (c[2] - c[0]) + b * (c[4] - c[2]) + d * (c[6] - c[4]);
    const double dy = a * (c[3] - c[1]) + b * (c[5] - c[3]) + d * (c[7] - c[5]);
    return std::hypot(dx, dy);
}

namespace {
struct Rule16 {
    std::vector<double> x, w;
    Rule16() { gauss_legendre(16, x, w); }
};
const Rule16& rule16() {
    static Rule16 r;
    return r;
}
double gl16(const double* c, double a, double b) {
    const Rule16& r = rule16();
    const double h = 0.5 * (b - a), m = 0.5 * (a + b);
    double acc = 0.0;
    for (int i = 0; i < 16; ++i) acc += r.w[i] * speed(c, m + h * r.x[i]);
    return acc * h;
}
void refine(const double* c, double a, double b, double whole, double tol, int depth,
            std::vector<double>& t, std::vector<double>& len) {
    const double m = 0.5 * (a + b);
    const double l = gl16(c, a, m), r = gl16(c, m, b);
    if (std::fabs(l + r - whole) <= tol || depth >= 48) {
        t.push_back(m);
        len.push_back(l);
        t.push_back(b);
        len.push_back(r);
        return;
    }
    refine(c, a, m, l, tol, depth + 1, t, len);
    refine(c, m, b, r, tol, depth + 1, t, len);
}
}  // namespace

// Cumulative arc-length table: adaptive composite 16-point GL on [0, 1].
ArcTable build_arc_table(const double* c) {
    double est = 0.0;
    for (int k = 0; k < 32; ++k) est += gl16(c, k / 32.0, (k + 1) / 32.0);
    ArcTable tab;
    tab.t.push_back(0.0);
    std::vector<double> lens;
    const double tol = 1e-16 * std::max(est, 1e-300);
    for (int k = 0; k < 32; ++k) {
        const double a = k / 32.0, b = (k + 1) / 32.0;
        refine(c, a, b, gl16(c, a, b), tol, 0, tab.t, lens);
    }
    tab.cum.assign(tab.t.size(), 0.0);
    for (size_t k = 0; k < lens.size(); ++k) tab.cum[k + 1] = tab.cum[k] + lens[k];
    tab.total = tab.cum.back();
    return tab;
}

// Parameter t with L(t) = T: Newton's method t <- t - (L(t) - T) / |B'(t)|
// (App. B) inside the table interval that brackets T, with bisection as a
// safeguard.  L(t) = cum[k] + GL16 on [t_k, t].
double param_at_length(const double* c, const ArcTable& tab, double T) {
    if (T <= 0.0) return 0.0;
    if (T >= tab.total) return 1.0;
    size_t k = std::upper_bound(tab.cum.begin(), tab.cum.end(), T) - tab.cum.begin();
    k = std::min(std::max<size_t>(k, 1), tab.cum.size() - 1) - 1;
    double lo = tab.t[k], hi = tab.t[k + 1];
    const double base = tab.cum[k];
    double span = tab.cum[k + 1] - base;
    double t = lo + (span > 0 ? (T - base) / span : 0.5) * (hi - lo);
    const double tol = 2e-15 * tab.total;
    for (int it = 0; it < 80; ++it) {
        const double f = base + gl16(c, tab.t[k], t) - T;
        if (std::fabs(f) <= tol) break;
        if (f > 0) hi = t; else lo = t;
        const double d = speed(c, t);
        double tn = d > 0 ? t - f / d : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (tn == t) break;
        t = tn;
    }
    return t;
}

// Lagrange basis of the g GL roots evaluated at the arc-length midpoints
// taubar_j = -1 + (2j+1)/s of the s segments: the matrix Pbar Pring^-1 of
// Eq. coefs_interp / Eq. legendre_poly written in its Lagrange form.
std::vector<double> interp_matrix(int g, int s) {
    std::vector<double> x, w;
    gauss_legendre(g, x, w);
    std::vector<double> pi((size_t)s * g, 1.0);
    for (int j = 0; j < s; ++j) {
        const double tb = -1.0 + (2.0 * j + 1.0) / s;
        for (int i = 0; i < g; ++i) {
            double v = 1.0;
            for (int m = 0; m < g; ++m)
                if (m != i) v *= (tb - x[m]) / (x[i] - x[m]);
            pi[(size_t)j * g + i] = v;
        }
    }
    return pi;
}

static void check_finite(const double* v, size_t n, const char* what) {
    for (size_t i = 0; i < n; ++i)
        DC_REQUIRE(std::isfinite(v[i]), std::string("non-finite value in ") + what);
}

void discretize(const double* ctrl, int n_curves, int P, int g, int s, Geometry& G) {
    DC_REQUIRE(n_curves > 0, "n_curves must be positive");
    DC_REQUIRE(P >= 1 && g >= 1 && s >= g, "need P >= 1, g >= 1 and s >= g");
    check_finite(ctrl, (size_t)n_curves * 8, "ctrl");
    G.n_curves = n_curves;
    G.P = P;
    G.g = g;
    G.s = s;
    G.N = n_curves * P * g;
    G.S = n_curves * P * s;
    std::vector<double> xg, wg;
    gauss_legendre(g, xg, wg);
    G.gl_x = xg;
    G.node_x.resize(G.N);
    G.node_y.resize(G.N);
    G.node_lam.resize(G.N);
    G.node_self.resize(G.N);
    G.node_tstar.resize(G.N);
    G.seg_x0.resize(G.S);
    G.seg_y0.resize(G.S);
    G.seg_x1.resize(G.S);
    G.seg_y1.resize(G.S);
    G.seg_ell.resize(G.S);
    G.seg_kappa.resize(G.S);
    G.curve_len.resize(n_curves);
    std::vector<int> jloc(g);
    std::vector<double> tstar(g);
    for (int k = 0; k < g; ++k) {
        // self segment: tau_j <= x_k < tau_{j+1}, tau_j = -1 + 2j/s (App. C.1)
        int j = (int)std::floor((xg[k] + 1.0) * s / 2.0);
        j = std::min(std::max(j, 0), s - 1);
        jloc[k] = j;
        tstar[k] = (xg[k] - (-1.0 + 2.0 * j / s)) / (2.0 / s);
    }
    std::vector<double> ex(s + 1), ey(s + 1);
    for (int c = 0; c < n_curves; ++c) {
        const double* cc = ctrl + (size_t)c * 8;
        ArcTable tab = build_arc_table(cc);
        DC_REQUIRE(tab.total > 0.0 && std::isfinite(tab.total), "zero-length curve");
        G.curve_len[c] = tab.total;
        const double L = tab.total;
        for (int p = 0; p < P; ++p) {
            const int panel = c * P + p;
            for (int k = 0; k < g; ++k) {
                const double lam = (p + 0.5 * (xg[k] + 1.0)) / P;
                const double t = param_at_length(cc, tab, L * lam);
                const int i = panel * g + k;
                bezier(cc, t, G.node_x[i], G.node_y[i]);
                G.node_lam[i] = lam;
                G.node_self[i] = panel * s + jloc[k];
                G.node_tstar[i] = tstar[k];
            }
            for (int j = 0; j <= s; ++j) {
                const double t = param_at_length(cc, tab, L * ((p + (double)j / s) / P));
                bezier(cc, t, ex[j], ey[j]);
            }
            const double ell = L / ((double)P * s);
            for (int j = 0; j < s; ++j) {
                const int q = panel * s + j;
                G.seg_x0[q] = ex[j];
                G.seg_y0[q] = ey[j];
                G.seg_x1[q] = ex[j + 1];
                G.seg_y1[q] = ey[j + 1];
                const double chord = std::hypot(ex[j + 1] - ex[j], ey[j + 1] - ey[j]);
                DC_REQUIRE(chord > 0.0, "degenerate (zero-length) chord segment");
                G.seg_ell[q] = ell;
                G.seg_kappa[q] = ell / chord;
            }
        }
    }
    G.Pi = interp_matrix(g, s);
    G.panel_curve.resize((size_t)n_curves * P);
    G.panel_lo.resize((size_t)n_curves * P);
    G.panel_hi.resize((size_t)n_curves * P);
    for (int c = 0; c < n_curves; ++c)
        for (int p = 0; p < P; ++p) {
            G.panel_curve[(size_t)c * P + p] = c;
            G.panel_lo[(size_t)c * P + p] = (double)p / P;
            G.panel_hi[(size_t)c * P + p] = (double)(p + 1) / P;
        }
}

void discretize_panels(const double* ctrl, int n_curves, const int* pc, const double* lo,
                       const double* hi, int n_panels, int g, int s, Geometry& G) {
    DC_REQUIRE(n_curves > 0 && n_panels > 0, "need curves and panels");
    DC_REQUIRE(g >= 1 && s >= g, "need g >= 1 and s >= g");
    DC_REQUIRE((long long)n_panels * s < (1LL << 31), "too many segments");
    check_finite(ctrl, (size_t)n_curves * 8, "ctrl");
    check_finite(lo, (size_t)n_panels, "panel_lo");
    check_finite(hi, (size_t)n_panels, "panel_hi");
    for (int k = 0; k < n_panels; ++k) {
        DC_REQUIRE(pc[k] >= 0 && pc[k] < n_curves, "panel curve out of range");
        DC_REQUIRE(lo[k] >= 0.0 && hi[k] <= 1.0 && lo[k] < hi[k], "panel range outside [0, 1]");
        if (k > 0) DC_REQUIRE(pc[k] > pc[k - 1] || (pc[k] == pc[k - 1] && lo[k] >= hi[k - 1]),
                              "panels must be listed curve by curve, in order along each");
    }
    G.n_curves = n_curves;
    G.P = 0;
    G.g = g;
    G.s = s;
    G.N = n_panels * g;
    G.S = n_panels * s;
    std::vector<double> xg, wg;
    gauss_legendre(g, xg, wg);
    G.gl_x = xg;
    G.node_x.resize(G.N);
    G.node_y.resize(G.N);
    G.node_lam.resize(G.N);
    G.node_self.resize(G.N);
    G.node_tstar.resize(G.N);
    G.seg_x0.resize(G.S);
    G.seg_y0.resize(G.S);
    G.seg_x1.resize(G.S);
    G.seg_y1.resize(G.S);
    G.seg_ell.resize(G.S);
    G.seg_kappa.resize(G.S);
    G.curve_len.assign(n_curves, 0.0);
    G.panel_curve.assign(pc, pc + n_panels);
    G.panel_lo.assign(lo, lo + n_panels);
    G.panel_hi.assign(hi, hi + n_panels);
    std::vector<int> jloc(g);
    std::vector<double> tstar(g);
    for (int k = 0; k < g; ++k) {
        // self segment: tau_j <= x_k < tau_{j+1}, tau_j = -1 + 2j/s (App. C.1)
        int j = (int)std::floor((xg[k] + 1.0) * s / 2.0);
        j = std::min(std::max(j, 0), s - 1);
        jloc[k] = j;
        tstar[k] = (xg[k] - (-1.0 + 2.0 * j / s)) / (2.0 / s);
    }
    std::vector<double> ex(s + 1), ey(s + 1);
    int cur = -1;
    ArcTable tab;
    for (int panel = 0; panel < n_panels; ++panel) {
        const int c = pc[panel];
        const double* cc = ctrl + (size_t)c * 8;
        if (c != cur) {
            tab = build_arc_table(cc);
            DC_REQUIRE(tab.total > 0.0 && std::isfinite(tab.total), "zero-length curve");
            G.curve_len[c] = tab.total;
            cur = c;
        }
        const double L = tab.total, a = lo[panel], w = hi[panel] - lo[panel];
        for (int k = 0; k < g; ++k) {
            const double lam = a + w * (0.5 * (xg[k] + 1.0));
            const double t = param_at_length(cc, tab, L * lam);
            const int i = panel * g + k;
            bezier(cc, t, G.node_x[i], G.node_y[i]);
            G.node_lam[i] = lam;
            G.node_self[i] = panel * s + jloc[k];
            G.node_tstar[i] = tstar[k];
        }
        for (int j = 0; j <= s; ++j) {
            const double t = param_at_length(cc, tab, L * (a + w * ((double)j / s)));
            bezier(cc, t, ex[j], ey[j]);
        }
        const double ell = L * w / s;
        for (int j = 0; j < s; ++j) {
            const int q = panel * s + j;
            G.seg_x0[q] = ex[j];
            G.seg_y0[q] = ey[j];
            G.seg_x1[q] = ex[j + 1];
            G.seg_y1[q] = ey[j + 1];
            const double chord = std::hypot(ex[j + 1] - ex[j], ey[j + 1] - ey[j]);
            DC_REQUIRE(chord > 0.0, "degenerate (zero-length) chord segment");
            G.seg_ell[q] = ell;
            G.seg_kappa[q] = ell / chord;
        }
    }
    for (int c = 0; c < n_curves; ++c)
        if (G.curve_len[c] == 0.0) {
            const ArcTable t2 = build_arc_table(ctrl + (size_t)c * 8);
            G.curve_len[c] = t2.total;
        }
    G.Pi = interp_matrix(g, s);
}

// Colour piecewise linear in normalised arc length through stops at
// lambda = k/(n-1).
static double colour(const double* stops, int n, int ch, double lam) {
    double u = lam * (n - 1);
    int k = (int)std::floor(u);
    k = std::min(std::max(k, 0), n - 2);
    const double f = u - k;
    return (1.0 - f) * stops[k * 3 + ch] + f * stops[(k + 1) * 3 + ch];
}

void boundary_from_stops(const Geometry& G, const double* left, const double* right,
                         int n_stops, std::vector<double>& up, std::vector<double>& um) {
    DC_REQUIRE(n_stops >= 2, "need at least two colour stops per side");
    check_finite(left, (size_t)G.n_curves * n_stops * 3, "left_rgb");
    check_finite(right, (size_t)G.n_curves * n_stops * 3, "right_rgb");
    up.assign((size_t)3 * G.N, 0.0);
    um.assign((size_t)3 * G.N, 0.0);
    for (int i = 0; i < G.N; ++i) {
        const int c = G.panel_curve[i / G.g];
        for (int ch = 0; ch < 3; ++ch) {
            up[(size_t)ch * G.N + i] = colour(left + (size_t)c * n_stops * 3, n_stops, ch, G.node_lam[i]);
            um[(size_t)ch * G.N + i] = colour(right + (size_t)c * n_stops * 3, n_stops, ch, G.node_lam[i]);
        }
    }
}

}  // namespace dc

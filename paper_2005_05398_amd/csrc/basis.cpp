// 1D Hermite spline bases and Gauss collocation points (host, FP64).
//
// Paper Sec. 3.1: local basis functions on [0, R] with zero Dirichlet
// conditions at the x and y endpoints, and on [-1, 1] for z; Sec. 4: Hermite
// splines with three functions per node (quintic S_5^3; cubic uses two),
// support on two adjacent intervals, node maps, collocation at Gaussian points.
//
// Closures (the paper does not state how the collocation system is squared):
//   x, y degree 3: n = 2K, 2 Gauss points per interval.
//   x, y degree 5: n = 3K + 1, 3 Gauss points per interval, 4 in the first.
//   z degree 3:   n = 2K + 2, 2 per interval, 1 extra in each end interval.
//   z degree 5:   n = 3K + 3, 3 per interval, 1 extra in each end interval and
//                 1 in the middle interval (K odd) or at the middle node (K even).
//   z halved to [0, 1] (a component of definite parity about z = 0, Sec. 2,
//   "Permutational symmetry"): the full basis's nodes and points in [0, 1],
//   the functions at z = 0 restricted to the parity.
// The function of derivative order d at a node carries the factor 1/hbar^d,
// hbar = R/K (x, y) or 2/K (z), so its coefficient is hbar^d psi^(d)(node).
#include <algorithm>
#include <cmath>

#include "fm_internal.h"

namespace fm {

namespace {

// Gauss-Legendre nodes on [-1, 1] by Newton's iteration on P_n.
std::vector<double> gauss_nodes(int n) {
    std::vector<double> x(n);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        x[i] = t;
    }
    std::sort(x.begin(), x.end());
    return x;
}

// Hermite shape functions on [0, 1]: value of the deriv-th s-derivative of
// the function attached to end e (0: s = 0, 1: s = 1) with derivative order d.
double shape(int q, int e, int d, int deriv, double s) {
    const double s2 = s * s, s3 = s2 * s, s4 = s3 * s, s5 = s4 * s;
    if (q == 2) {
        if (e == 0 && d == 0) return deriv == 0 ? 1 - 3 * s2 + 2 * s3 : deriv == 1 ? -6 * s + 6 * s2 : -6 + 12 * s;
        if (e == 0 && d == 1) return deriv == 0 ? s - 2 * s2 + s3 : deriv == 1 ? 1 - 4 * s + 3 * s2 : -4 + 6 * s;
        if (e == 1 && d == 0) return deriv == 0 ? 3 * s2 - 2 * s3 : deriv == 1 ? 6 * s - 6 * s2 : 6 - 12 * s;
        return deriv == 0 ? -s2 + s3 : deriv == 1 ? -2 * s + 3 * s2 : -2 + 6 * s;
    }
    if (e == 0) {
        if (d == 0) return deriv == 0 ? 1 - 10 * s3 + 15 * s4 - 6 * s5
                         : deriv == 1 ? -30 * s2 + 60 * s3 - 30 * s4 : -60 * s + 180 * s2 - 120 * s3;
        if (d == 1) return deriv == 0 ? s - 6 * s3 + 8 * s4 - 3 * s5
                         : deriv == 1 ? 1 - 18 * s2 + 32 * s3 - 15 * s4 : -36 * s + 96 * s2 - 60 * s3;
        return deriv == 0 ? 0.5 * (s2 - 3 * s3 + 3 * s4 - s5)
             : deriv == 1 ? 0.5 * (2 * s - 9 * s2 + 12 * s3 - 5 * s4) : 0.5 * (2 - 18 * s + 36 * s2 - 20 * s3);
    }
    if (d == 0) return deriv == 0 ? 10 * s3 - 15 * s4 + 6 * s5
                     : deriv == 1 ? 30 * s2 - 60 * s3 + 30 * s4 : 60 * s - 180 * s2 + 120 * s3;
    if (d == 1) return deriv == 0 ? -4 * s3 + 7 * s4 - 3 * s5
                     : deriv == 1 ? -12 * s2 + 28 * s3 - 15 * s4 : -24 * s + 84 * s2 - 60 * s3;
    return deriv == 0 ? 0.5 * (s3 - 2 * s4 + s5)
         : deriv == 1 ? 0.5 * (3 * s2 - 8 * s3 + 5 * s4) : 0.5 * (6 * s - 24 * s2 + 20 * s3);
}

}  // namespace

std::string Basis1D::init(const fm_dim &d, bool is_z) {
    degree = d.degree;
    n = d.n;
    if (degree != 3 && degree != 5) return "degree must be 3 or 5";
    q = (degree + 1) / 2;
    std::vector<int> counts;
    int extra_node = -1;
    if (!is_z) {
        dirichlet = true;
        if (!(d.R > 0) || !std::isfinite(d.R)) return "R must be positive";
        R = d.R;
        lo = 0.0;
        if (degree == 3) {
            if (n < 2 || n % 2) return "cubic x/y basis needs an even n >= 2";
            K = n / 2;
            counts.assign(K, 2);
        } else {
            if (n < 4 || n % 3 != 1) return "quintic x/y basis needs n = 3K + 1";
            K = (n - 1) / 3;
            counts.assign(K, 3);
            counts[0] = 4;
        }
    } else {
        dirichlet = false;
        R = 2.0;
        lo = -1.0;
        if (degree == 3) {
            if (n < 4 || n % 2) return "cubic z basis needs an even n >= 4";
            K = (n - 2) / 2;
        } else {
            if (n < 6 || n % 3) return "quintic z basis needs n = 3K + 3";
            K = n / 3 - 1;
        }
        counts.assign(K, q);
        counts[0] += 1;
        counts[K - 1] += 1;
        if (degree == 5) {
            if (K % 2) counts[(K - 1) / 2] += 1;
            else extra_node = K / 2;
        }
    }
    if (K > 4096) return "too many intervals";
    hbar = R / K;
    nodes.resize(K + 1);
    for (int i = 0; i <= K; ++i) {
        double u = double(i) / K;
        double t;
        if (!is_z) {
            switch (d.map) {
                case FM_MAP_UNIFORM: t = R * u; break;
                case FM_MAP_QUADRATIC: t = R * u * u; break;
                case FM_MAP_POW: t = 4.0 * (std::pow(1.0 + R / 4.0, u) - 1.0); break;
                default: return "x/y map must be uniform, quadratic or pow";
            }
        } else {
            double v = -1.0 + 2.0 * u;
            switch (d.map) {
                case FM_MAP_SIN: t = std::sin(M_PI * v / 2.0); break;
                case FM_MAP_UNIFORM: t = v; break;
                default: return "z map must be sin or uniform";
            }
        }
        nodes[i] = t;
    }
    if (is_z) { nodes[0] = -1.0; nodes[K] = 1.0; }
    else { nodes[0] = 0.0; nodes[K] = R; }
    for (int i = 0; i < K; ++i)
        if (!(nodes[i + 1] > nodes[i])) return "node map is not increasing";
    points.clear();
    for (int m = 0; m < K; ++m) {
        std::vector<double> g = gauss_nodes(counts[m]);
        double a = nodes[m], b = nodes[m + 1];
        for (double gi : g) points.push_back(0.5 * (a + b) + 0.5 * (b - a) * gi);
    }
    if (extra_node >= 0) points.push_back(nodes[extra_node]);
    std::sort(points.begin(), points.end());
    if ((int)points.size() != n) return "internal: point count";
    idx.assign(size_t(n) * MAXR, -1);
    for (int k = 0; k < 3; ++k) val[k].assign(size_t(n) * MAXR, 0.0);
    for (int p = 0; p < n; ++p) {
        int g[MAXR];
        double v[MAXR];
        for (int k = 0; k < 3; ++k) {
            eval_local(points[p], k, g, v);
            for (int sl = 0; sl < 2 * q; ++sl) {
                idx[size_t(p) * MAXR + sl] = g[sl];
                val[k][size_t(p) * MAXR + sl] = g[sl] >= 0 ? v[sl] : 0.0;
            }
        }
    }
    return "";
}

std::string Basis1D::init_half(const fm_dim &d, int sigma) {
    degree = d.degree;
    if (degree != 3 && degree != 5) return "degree must be 3 or 5";
    q = (degree + 1) / 2;
    int Kf;
    if (degree == 3) {
        if (d.n < 4 || d.n % 2) return "cubic z basis needs an even n >= 4";
        Kf = (d.n - 2) / 2;
    } else {
        if (d.n < 6 || d.n % 3) return "quintic z basis needs n = 3K + 3";
        Kf = d.n / 3 - 1;
    }
    if (Kf % 2) return "a z basis halved to [0, 1] needs an even number of intervals (z = 0 a node)";
    if (sigma != 1 && sigma != -1) return "parity must be +1 or -1";
    half = sigma;
    dirichlet = false;
    K = Kf / 2;
    R = 1.0;
    lo = 0.0;
    hbar = 1.0 / K;                              // = 2 / Kf, the full basis's hbar
    // node 0 keeps the orders of the parity: even functions have odd derivatives
    // zero there, odd functions even ones
    int kept0 = 0;
    for (int o = 0; o < q; ++o) kept0 += ((o % 2 == 0) == (sigma == 1)) ? 1 : 0;
    n = kept0 + K * q;
    nodes.resize(K + 1);
    for (int i = 0; i <= K; ++i) {
        const double u = double(i) / K;
        switch (d.map) {
            case FM_MAP_SIN: nodes[i] = std::sin(M_PI * u / 2.0); break;
            case FM_MAP_UNIFORM: nodes[i] = u; break;
            default: return "z map must be sin or uniform";
        }
    }
    nodes[0] = 0.0;
    nodes[K] = 1.0;
    // the full basis's points in [0, 1]: q Gauss points per interval, one more
    // in the end interval at z = 1, and (quintic) the full basis's node point
    // z = 0, which only even functions keep as a collocation point
    std::vector<int> counts(K, q);
    counts[K - 1] += 1;
    points.clear();
    for (int m = 0; m < K; ++m) {
        std::vector<double> g = gauss_nodes(counts[m]);
        const double a = nodes[m], b = nodes[m + 1];
        for (double gi : g) points.push_back(0.5 * (a + b) + 0.5 * (b - a) * gi);
    }
    if (degree == 5 && sigma == 1) points.push_back(0.0);
    std::sort(points.begin(), points.end());
    if ((int)points.size() != n) return "internal: half-basis point count";
    idx.assign(size_t(n) * MAXR, -1);
    for (int k = 0; k < 3; ++k) val[k].assign(size_t(n) * MAXR, 0.0);
    for (int p = 0; p < n; ++p) {
        int g[MAXR];
        double v[MAXR];
        for (int k = 0; k < 3; ++k) {
            eval_local(points[p], k, g, v);
            for (int sl = 0; sl < 2 * q; ++sl) {
                idx[size_t(p) * MAXR + sl] = g[sl];
                val[k][size_t(p) * MAXR + sl] = g[sl] >= 0 ? v[sl] : 0.0;
            }
        }
    }
    return "";
}

int Basis1D::global_index(int m, int d) const {
    if (half) {
        // node 0 keeps the orders of the parity, numbered first; then q per node
        auto kept = [&](int o) { return (o % 2 == 0) == (half == 1); };
        if (m == 0) {
            if (!kept(d)) return -1;
            int r = 0;
            for (int o = 0; o < d; ++o) r += kept(o) ? 1 : 0;
            return r;
        }
        int k0 = 0;
        for (int o = 0; o < q; ++o) k0 += kept(o) ? 1 : 0;
        return k0 + (m - 1) * q + d;
    }
    if (dirichlet && d == 0 && (m == 0 || m == K)) return -1;
    int g = m * q + d - (dirichlet ? 1 : 0);
    if (dirichlet && m == K) g -= 1;            // skip the dropped value function at node K
    return g;
}

int Basis1D::interval(double t) const {
    // the last m with nodes[m] <= t, clamped to [0, K-1]
    int m = int(std::upper_bound(nodes.begin(), nodes.end(), t) - nodes.begin()) - 1;
    return std::min(std::max(m, 0), K - 1);
}

void Basis1D::eval_local(double t, int deriv, int *gidx, double *v) const {
    int m = interval(t);
    double h = nodes[m + 1] - nodes[m];
    double s = (t - nodes[m]) / h;
    for (int e = 0; e < 2; ++e)
        for (int d = 0; d < q; ++d) {
            int sl = e * q + d;
            double f = std::pow(h / hbar, d) / std::pow(h, deriv);
            v[sl] = shape(q, e, d, deriv, s) * f;
            if (gidx) gidx[sl] = global_index(m + e, d);
        }
}

std::vector<double> Basis1D::dense(int deriv) const {
    std::vector<double> B(size_t(n) * n, 0.0);
    for (int p = 0; p < n; ++p)
        for (int sl = 0; sl < 2 * q; ++sl) {
            int g = idx[size_t(p) * MAXR + sl];
            if (g >= 0) B[size_t(p) * n + g] += val[deriv][size_t(p) * MAXR + sl];
        }
    return B;
}

}  // namespace fm

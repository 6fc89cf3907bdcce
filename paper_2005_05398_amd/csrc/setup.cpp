// Problem set-up (host, FP64) and upload of every energy-independent array.
//
// Paper Sec. 2.1: reduced masses, eq. (JacobiTrans) coefficients, Coulomb pair
// potentials, the Merkuriev split (eq. (split3b)) with the cut-off of
// eq. (Mcutoff0).  Sec. 2.2: x_b, y_b, z_b(x_a, y_a, z_a), F functions.
// Sec. 3.1: Vhat_a.  Sec. 3.2: the pencils whose generalized eigenvectors make
// the tensor-trick preconditioner.
//
// The block-Jacobi preconditioner (variant 1) is the exact inverse of the
// separable block L_alpha of eq. (FM-fin), M'-block by M'-block (the M' +- 1
// blocks are left out).  For a block M' the z pencil (d_z^{M'} operator, S_z)
// is diagonalised first (eq. (z-dec)); with mu_k = -lambda~_{z,k} each z mode k
// then leaves the 2D operator (A_x^k (x) S_y + S_x (x) A_y^k - E S_x (x) S_y)
// with
//   A_x^k = -D_x + mu_k X_r2 S_x + V_a S_x,
//   A_y^k = -D_y + (J(J+1) - 2M'^2 + mu_k) Y_r2 S_y + Vhat_a S_y,
// whose inverse follows from eq. (MDA) with the pencils (A_x^k, S_x) and
// (A_y^k, S_y).  The coupled preconditioner (variant 2, coupled.cpp) has the
// same x-y structure with other coefficients per slot and a joint z matrix.
// All factors are independent of E; only the final divide by
// lambda_x + lambda_y - E sees the energy.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "fm_problem.h"

namespace fm {

namespace {

double factorial(int n) {
    double f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// Coefficients of d^J_{M M'}(w) as a homogeneous polynomial of degree 2J in
// (cos(w/2), sin(w/2)): d = sum_p f[p] c^p s^(2J-p), Wigner's explicit sum.
void wigner_poly(int J, int M, int Mp, std::vector<double> &f) {
    f.assign(2 * J + 1, 0.0);
    if (std::abs(M) > J || std::abs(Mp) > J) return;
    double pref = std::sqrt(factorial(J + M) * factorial(J - M) * factorial(J + Mp) * factorial(J - Mp));
    for (int k = 0; k <= 2 * J; ++k) {
        int a1 = J + Mp - k, a2 = k, a3 = M - Mp + k, a4 = J - M - k;
        if (a1 < 0 || a2 < 0 || a3 < 0 || a4 < 0) continue;
        double den = factorial(a1) * factorial(a2) * factorial(a3) * factorial(a4);
        double sgn = ((M - Mp + k) % 2 == 0) ? 1.0 : -1.0;
        int pc = 2 * J + Mp - M - 2 * k;
        f[pc] += pref * sgn / den;
    }
}

}  // namespace

std::string setup_problem(fm_problem *p) {
    const fm_problem_desc &d = p->desc;
    if (d.tau != 1 && d.tau != -1) return "tau must be +1 or -1";
    if (d.J < 0 || d.J > MAXM - 1) return "J must be between 0 and 15 (at most 16 M' blocks)";
    p->M0 = (1 - d.tau) / 2;
    p->nM = d.J - p->M0 + 1;
    if (p->nM < 1) return "no M' blocks for this J, tau";
    if (p->nM > MAXM) return "too many M' blocks";
    for (int a = 0; a < 3; ++a) {
        if (!(d.mass[a] > 0) || !std::isfinite(d.mass[a])) return "masses must be positive";
        if (!std::isfinite(d.charge[a])) return "charges must be finite";
    }
    if (!(d.x0 > 0) || !(d.nu > 0) || !(d.y0 > 0)) return "cut-off parameters must be positive";
    if (d.vhat != 0) return "only vhat = 0 is defined";
    if (d.precond != 0 && d.precond != FM_PREC_BLOCK_JACOBI && d.precond != FM_PREC_COUPLED)
        return "precond must be FM_PREC_BLOCK_JACOBI or FM_PREC_COUPLED";
    p->variant = d.precond == FM_PREC_COUPLED ? 2 : 1;
    if (!std::isfinite(d.mode_fit_tol)) return "mode_fit_tol must be finite";
    p->mode_fit_tol = d.mode_fit_tol > 0 ? d.mode_fit_tol : FM_DEFAULT_MODE_FIT_TOL;
    if (d.exchange != 0 && d.exchange != 1 && d.exchange != -1 && d.exchange != 3)
        return "exchange must be 0, +1, -1 or 3";
    p->exchange = d.exchange;
    if (d.exchange != 0) {
        auto same = [](const fm_dim &u, const fm_dim &v) {
            return u.degree == v.degree && u.n == v.n && u.R == v.R && u.map == v.map;
        };
        if (d.mass[0] != d.mass[1] || d.charge[0] != d.charge[1])
            return "exchange symmetry needs particles 1 and 2 with equal masses and charges";
        if (!same(d.x[0], d.x[1]) || !same(d.y[0], d.y[1]) || !same(d.z[0], d.z[1]))
            return "exchange symmetry needs identical bases for components 1 and 2";
        if (d.exchange == 3) {
            if (d.mass[2] != d.mass[0] || d.charge[2] != d.charge[0])
                return "three identical particles need equal masses and charges";
            if (!same(d.x[0], d.x[2]) || !same(d.y[0], d.y[2]) || !same(d.z[0], d.z[2]))
                return "three identical particles need identical bases for all components";
        }
    }
    if (d.zhalf != 0 && d.zhalf != 1) return "zhalf must be 0 or 1";
    p->zhalf = d.zhalf;
    p->zsigma = 1;
    if (d.zhalf) {
        if (d.exchange != 1 && d.exchange != -1) return "zhalf needs the exchange symmetry of two particles (+1 or -1)";
        if (p->nM != 1) return "zhalf needs one M' block (its parity (-1)^{M'} p fixes one z basis)";
        if (d.precond == FM_PREC_COUPLED) return "zhalf is for the block-Jacobi preconditioner (n_M = 1)";
        p->zsigma = d.exchange * ((p->M0 & 1) ? -1 : 1);
    }
    for (int a = 0; a < 3; ++a) {
        std::string e = p->bx[a].init(d.x[a], false);
        if (e.empty()) e = p->by[a].init(d.y[a], false);
        if (e.empty()) e = (a == 2 && p->zhalf) ? p->bz[a].init_half(d.z[a], p->zsigma) : p->bz[a].init(d.z[a], true);
        if (!e.empty()) return "component " + std::to_string(a) + ": " + e;
    }
    // kinematics
    const double *m = d.mass;
    double M = m[0] + m[1] + m[2];
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        p->mu[a] = m[b] * m[c] / (m[b] + m[c]);
        p->mu_abc[a] = m[a] * (m[b] + m[c]) / M;
        p->zz[a] = d.charge[b] * d.charge[c];
    }
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            if (a == b) { p->crot[b][a] = 1; p->srot[b][a] = 0; continue; }
            double c = -std::sqrt(m[b] * m[a] / ((M - m[b]) * (M - m[a])));
            double sgn = ((b - a) % 2 == 0 ? 1.0 : -1.0) * (a > b ? 1.0 : -1.0);
            p->crot[b][a] = c;
            p->srot[b][a] = sgn * std::sqrt(std::max(0.0, 1.0 - c * c));
        }
    // sizes
    long long off = 0;
    for (int a = 0; a < 3; ++a) {
        p->npts[a] = p->absent(a) ? 0 : (long long)p->bz[a].n * p->bx[a].n * p->by[a].n;
        p->off[a] = off;
        off += p->npts[a] * p->nM;
    }
    p->N = off;
    if (p->N > (1LL << 31)) return "problem too large";

    // angular constants
    ProblemDev &pd = p->pd;
    std::memset(&pd, 0, sizeof(pd));
    pd.nM = p->nM;
    pd.J = d.J;
    pd.tau = d.tau;
    pd.M0 = p->M0;
    pd.N = p->N;
    int J = d.J;
    for (int i = 0; i < p->nM; ++i) {
        int Mp = p->M0 + i;
        double lp = std::sqrt(std::max(0.0, double(J * (J + 1) - Mp * (Mp + 1))));
        double lm = std::sqrt(std::max(0.0, double(J * (J + 1) - Mp * (Mp - 1))));
        pd.lhp[i] = lp * std::sqrt(1.0 + (Mp == 0));
        pd.lhm[i] = lm * std::sqrt(1.0 + (Mp == 1));
    }
    // coupling weight table: G[iM'][iM''][p], weight = sum_p G c^p s^(2J-p)
    pd.dlen = 2 * J + 1;
    if (p->nM * p->nM * pd.dlen > (int)(sizeof(pd.dcoef) / sizeof(double))) return "J too large";
    std::vector<double> f1, f2;
    for (int i = 0; i < p->nM; ++i)
        for (int k = 0; k < p->nM; ++k) {
            int Mp = p->M0 + i, Mpp = p->M0 + k;
            wigner_poly(J, Mpp, Mp, f1);
            wigner_poly(J, Mpp, -Mp, f2);
            double norm = 1.0 / std::sqrt(2.0 + 2.0 * (Mp == 0));
            double par = (Mp % 2 == 0) ? 1.0 : -1.0;
            double pre = (((Mpp - Mp) % 2 == 0) ? 1.0 : -1.0) * 2.0 / std::sqrt(2.0 + 2.0 * (Mpp == 0));
            for (int q = 0; q < pd.dlen; ++q)
                pd.dcoef[(i * p->nM + k) * pd.dlen + q] = pre * norm * (f1[q] + d.tau * par * f2[q]);
        }
    return "";
}

double coulomb(const fm_problem *p, int a, double x) { return std::sqrt(2.0 * p->mu[a]) * p->zz[a] / x; }

double cutoff(const fm_problem *p, double x, double y) {
    const fm_problem_desc &d = p->desc;
    double den = 1.0 + (std::isfinite(d.y0) ? y / d.y0 : 0.0);
    double arg = std::pow(x / d.x0, d.nu) / den;
    return 2.0 / (1.0 + std::exp(std::min(arg, 700.0)));
}

double vhat(const fm_problem *p, int a, double y) {
    const double *Z = p->desc.charge;
    int b = (a + 1) % 3, c = (a + 2) % 3;
    return Z[a] * (Z[b] + Z[c]) * std::sqrt(2.0 * p->mu_abc[a]) / (y + 1.0);
}

void rotate(double c, double s, double x, double y, double z, double &xb, double &yb, double &zb) {
    xb = std::sqrt(std::max(c * c * x * x + 2 * s * c * x * y * z + s * s * y * y, 0.0));
    yb = std::sqrt(std::max(s * s * x * x - 2 * s * c * x * y * z + c * c * y * y, 0.0));
    double den = xb * yb;
    zb = den > 0 ? (s * c * (y * y - x * x) + (c * c - s * s) * x * y * z) / den : 0.0;
    zb = std::min(1.0, std::max(-1.0, zb));
}

// All pencils of the preconditioner; fills the host factor arrays.
std::string build_factors(fm_problem *p, HostFactors &hf) {
    const fm_problem_desc &d = p->desc;
    int nM = p->nM, J = d.J;
    std::string err;
    std::mutex mu;
    hf.max_err = 0;
    for (int a = 0; a < 3; ++a) {
        if (p->absent(a)) continue;
        const Basis1D &bx = p->bx[a], &by = p->by[a], &bz = p->bz[a];
        int nx = bx.n, ny = by.n, nz = bz.n;
        HostComp &hc = hf.comp[a];
        hc.Wz.assign(size_t(nM) * 2 * nz * nz, 0.0);
        hc.Wx.assign(size_t(nM) * nz * 2 * nx * nx, 0.0);
        hc.Wy.assign(size_t(nM) * nz * 2 * ny * ny, 0.0);
        hc.lx.assign(size_t(nM) * nz * nx, 0.0);
        hc.lxi.assign(size_t(nM) * nz * nx, 0.0);
        hc.ly.assign(size_t(nM) * nz * ny, 0.0);
        hc.lyi.assign(size_t(nM) * nz * ny, 0.0);
        hc.tx.assign(size_t(nM) * nz * nx, 0);
        hc.ty.assign(size_t(nM) * nz * ny, 0);
        std::vector<double> Sz = bz.dense(0), D1z = bz.dense(1), D2z = bz.dense(2);
        std::vector<double> Sx = bx.dense(0), D2x = bx.dense(2);
        std::vector<double> Sy = by.dense(0), D2y = by.dense(2);
        // per slot: x pencil coefficient of X_r2 S_x, y pencil coefficient of Y_r2 S_y
        std::vector<double> cx(size_t(nM) * nz), cy(size_t(nM) * nz);
        std::vector<std::vector<double>> zWb(nM), zW(nM), zl(nM);
        std::vector<std::vector<char>> zres(nM);
        for (int iM = 0; iM < nM; ++iM) {
            int Mp = p->M0 + iM;
            std::vector<double> A1(size_t(nz) * nz);
            for (int i = 0; i < nz; ++i) {
                double z = bz.points[i];
                for (int j = 0; j < nz; ++j)
                    A1[size_t(i) * nz + j] = (1 - z * z) * D2z[size_t(i) * nz + j] -
                                             2.0 * (Mp + 1) * z * D1z[size_t(i) * nz + j] -
                                             double(Mp) * (Mp + 1) * Sz[size_t(i) * nz + j];
            }
            std::vector<double> Wb, W, lre, lim;
            std::vector<signed char> ty;
            double e = 0;
            std::string r = pencil_diag(nz, A1, Sz, Wb, W, lre, lim, ty, &e);
            if (!r.empty()) return "z pencil: " + r;
            for (int i = 0; i < nz; ++i)
                if (ty[i] != 0) return "z pencil has complex eigenvalues";
            hf.max_err = std::max(hf.max_err, e);
            if (p->variant == 2) {
                r = order_and_scale_z(bz, Mp, p->mode_fit_tol, Wb, W, lre, zres[iM]);
                if (!r.empty()) return "z pencil: " + r;
                zl[iM] = lre;
            }
            std::copy(Wb.begin(), Wb.end(), hc.Wz.begin() + size_t(iM) * 2 * nz * nz);
            std::copy(W.begin(), W.end(), hc.Wz.begin() + size_t(iM) * 2 * nz * nz + size_t(nz) * nz);
            for (int k = 0; k < nz; ++k) {
                const double mu_k = -lre[k];
                cx[size_t(iM) * nz + k] = mu_k;
                cy[size_t(iM) * nz + k] = double(J) * (J + 1) - 2.0 * Mp * Mp + mu_k;
            }
            zWb[iM].swap(Wb);
            zW[iM].swap(W);
        }
        if (p->variant == 2) {
            std::string r = coupled_slots(p, nz, zWb, zW, zl, zres, hc.Zj, cx, cy);
            if (!r.empty()) return r;
        }
        std::vector<double> Vx(nx), Vh(ny);
        for (int i = 0; i < nx; ++i) Vx[i] = coulomb(p, a, bx.points[i]);
        for (int j = 0; j < ny; ++j) Vh[j] = vhat(p, a, by.points[j]);
        // x and y pencils for every slot, in parallel
        int total = nM * nz;
        int nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        std::atomic<int> next(0);
        for (int t = 0; t < nthreads; ++t)
            pool.emplace_back([&]() {
                std::vector<double> A1x(size_t(nx) * nx), A1y(size_t(ny) * ny), Wb, W, lre, lim;
                std::vector<signed char> ty;
                for (;;) {
                    int job = next.fetch_add(1);
                    if (job >= total) break;
                    int iM = job / nz, k = job % nz;
                    for (int i = 0; i < nx; ++i) {
                        double x = bx.points[i];
                        double f = cx[job] / (x * x) + Vx[i];
                        for (int j = 0; j < nx; ++j)
                            A1x[size_t(i) * nx + j] = -D2x[size_t(i) * nx + j] + f * Sx[size_t(i) * nx + j];
                    }
                    for (int i = 0; i < ny; ++i) {
                        double y = by.points[i];
                        double f = cy[job] / (y * y) + Vh[i];
                        for (int j = 0; j < ny; ++j)
                            A1y[size_t(i) * ny + j] = -D2y[size_t(i) * ny + j] + f * Sy[size_t(i) * ny + j];
                    }
                    double ex = 0, ey = 0;
                    std::string r = pencil_diag(nx, A1x, Sx, Wb, W, lre, lim, ty, &ex);
                    if (r.empty()) {
                        size_t base = (size_t(iM) * nz + k) * 2 * nx * nx;
                        std::copy(Wb.begin(), Wb.end(), hc.Wx.begin() + base);
                        std::copy(W.begin(), W.end(), hc.Wx.begin() + base + size_t(nx) * nx);
                        size_t lb = (size_t(iM) * nz + k) * nx;
                        for (int i = 0; i < nx; ++i) {
                            hc.lx[lb + i] = lre[i];
                            hc.lxi[lb + i] = lim[i];
                            hc.tx[lb + i] = ty[i];
                        }
                        r = pencil_diag(ny, A1y, Sy, Wb, W, lre, lim, ty, &ey);
                        if (r.empty()) {
                            base = (size_t(iM) * nz + k) * 2 * ny * ny;
                            std::copy(Wb.begin(), Wb.end(), hc.Wy.begin() + base);
                            std::copy(W.begin(), W.end(), hc.Wy.begin() + base + size_t(ny) * ny);
                            lb = (size_t(iM) * nz + k) * ny;
                            for (int i = 0; i < ny; ++i) {
                                hc.ly[lb + i] = lre[i];
                                hc.lyi[lb + i] = lim[i];
                                hc.ty[lb + i] = ty[i];
                            }
                        } else {
                            r = "y pencil: " + r;
                        }
                    } else {
                        r = "x pencil: " + r;
                    }
                    std::lock_guard<std::mutex> g(mu);
                    if (!r.empty() && err.empty()) err = r;
                    hf.max_err = std::max(hf.max_err, std::max(ex, ey));
                }
            });
        for (auto &t : pool) t.join();
        if (!err.empty()) return err;
        // fields
        hc.P.resize(p->npts[a]);
        hc.Vs.resize(size_t(nx) * ny);
        for (int i = 0; i < nx; ++i)
            for (int j = 0; j < ny; ++j) {
                double x = bx.points[i], y = by.points[j];
                hc.Vs[size_t(i) * ny + j] = cutoff(p, x, y) * coulomb(p, a, x);
            }
        for (int kz = 0; kz < nz; ++kz)
            for (int i = 0; i < nx; ++i)
                for (int j = 0; j < ny; ++j) {
                    double z = bz.points[kz], x = bx.points[i], y = by.points[j];
                    double P = coulomb(p, a, x);
                    for (int b = 0; b < 3; ++b) {
                        if (b == a) continue;
                        double xb, yb, zb;
                        rotate(p->crot[b][a], p->srot[b][a], x, y, z, xb, yb, zb);
                        P += (1.0 - cutoff(p, xb, yb)) * coulomb(p, b, xb);
                    }
                    hc.P[(size_t(kz) * nx + i) * ny + j] = P;
                }
    }
    return "";
}

}  // namespace fm

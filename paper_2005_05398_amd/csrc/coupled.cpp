// Host set-up of the coupled L > 0 preconditioner (Sec. 3.2: the approximate
// matrix script-L_alpha with its M' +- 1 blocks; eq. (prop-eq); Appendix).
//
// The paper inverts script-L_alpha by z pencils per M', x pencils per
// l = M' + k, y pencils per (l, i_x) with the Y_r2 S_y mass (eq. (ops)) and a
// tridiagonal solve in M' per (l, i_x, i_y).  The y pencils there depend on
// the energy.  The same inverse follows from energy-independent factors by
// diagonalising, for each l, the n_l x n_l tridiagonal matrix T_l that couples
// the M' blocks sharing that l (n_l = number of M' with 0 <= l - M' < n_z):
//
//   T_l[M'][M']   = J(J+1) - 2M'^2 + l(l+1)
//   T_l[M'][M'+1] = -lambda-hat^{J,M'} lambda^{l,M'}
//   T_l[M'][M'-1] = -lambda-hat^{J,-M'} lambda^{l,-M'}
//
// (the entries of the P-blocks of Sec. 3.2 without the y eigenvalue).  T_l is
// similar to a symmetric matrix (the products of opposite off-diagonal
// entries are positive), so T_l = U_l diag(tau_{l,m}) U_l^-1 with real tau.
// After the z transform and the x transform of l, the system of (l, i_x) is
//   (A_y + (lambda_x - E) S_y) (x) I + (Y_r2 S_y) (x) T_l,
//   A_y = -D_y + Vhat S_y,
// and U_l^-1 splits it into one y operator A_y + tau_{l,m} Y_r2 S_y +
// (lambda_x - E) S_y per m: the pencil (A_y + tau_{l,m} Y_r2 S_y, S_y) then
// turns the whole inverse into the divide by lambda_x + lambda_y - E of the
// tensor trick.  Each (l, m) is one x-y "slot" with the x pencil of l and the
// y pencil of (l, m); the slots replace the (M', k) slices of the block-Jacobi
// variant one for one (sum_l n_l = n_M n_z), and the z transform and the M'
// mixing fold into one n_M n_z x n_M n_z matrix per direction.
//
// The substitution of eq. (prop-eq) (analytic eigenvalues, the bidiagonal
// Lambda^{M'+-}) presupposes z eigenvectors that represent g_l^{M'}; the
// pencil's highest modes do not (the spline space reproduces g_l^{M'} only up
// to its polynomial degree, roughly beyond), and a mode nearly orthogonal to
// its g would take a near-zero scale.  Such modes keep their computed
// eigenvalue and no M' coupling, one slot each, as in the block-Jacobi variant.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "fm_problem.h"

namespace fm {

namespace {

double lam_of(int j, int m) { return std::sqrt(std::max(0.0, double(j) * (j + 1) - double(m) * (m + 1))); }

}  // namespace

// g_l^M(z) of eq. (g-def): sqrt((2l+1)/2 (l-M)!/(l+M)!) P_l^M(z) / (1-z^2)^(M/2)
// with the Condon-Shortley phase, by the three-term recurrence in l of the
// normalised functions (starting value g_M^M = (-1)^M sqrt((2M+1)/2)
// prod_{i<=M} sqrt((2i-1)/(2i))).
double assoc_g(int l, int M, double z) {
    if (l < M) return 0.0;
    double g0 = std::sqrt((2.0 * M + 1.0) / 2.0);
    for (int i = 1; i <= M; ++i) g0 *= -std::sqrt((2.0 * i - 1.0) / (2.0 * i));
    if (l == M) return g0;
    double gm1 = g0, g = std::sqrt(2.0 * M + 3.0) * z * g0;
    for (int j = M + 2; j <= l; ++j) {
        const double jj = double(j) * j, mm = double(M) * M;
        const double a = std::sqrt((4.0 * jj - 1.0) / (jj - mm));
        const double b = std::sqrt(((j - 1.0) * (j - 1.0) - mm) * (2.0 * j + 1.0) / ((2.0 * j - 3.0) * (jj - mm)));
        const double gn = a * z * g - b * gm1;
        gm1 = g;
        g = gn;
    }
    return g;
}

// Orders the z pencil of block M' (Wbar, W row-major n x n, W's columns the
// eigenvectors) by ascending |lambda~| and fits column k to g_{M'+k}^{M'} at
// the collocation points in least squares.  Where the fit's relative residual
// is at most fit_tol the column takes the fitted scale (Wbar's row the inverse
// factor, which keeps Wbar S_z W = I) and the mode is marked resolved: the
// substitution of eq. (prop-eq) presupposes exactly these functions.  A mode
// that its eigenvector does not represent (the pencil's higher modes, beyond
// what the spline space reproduces) stays unscaled and unresolved.
std::string order_and_scale_z(const Basis1D &bz, int Mp, double fit_tol, std::vector<double> &Wb,
                              std::vector<double> &W, std::vector<double> &lre, std::vector<char> &resolved) {
    const int n = bz.n;
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) { return std::fabs(lre[i]) < std::fabs(lre[j]); });
    std::vector<double> W2(size_t(n) * n), Wb2(size_t(n) * n), l2(n);
    for (int c = 0; c < n; ++c) {
        const int o = ord[c];
        l2[c] = lre[o];
        for (int i = 0; i < n; ++i) {
            W2[size_t(i) * n + c] = W[size_t(i) * n + o];
            Wb2[size_t(c) * n + i] = Wb[size_t(o) * n + i];
        }
    }
    const std::vector<double> S = bz.dense(0);
    resolved.assign(n, 0);
    std::vector<double> v(n), g(n);
    for (int c = 0; c < n; ++c) {
        double gv = 0, vv = 0, gg = 0;
        for (int i = 0; i < n; ++i) {
            double t = 0;
            for (int j = 0; j < n; ++j) t += S[size_t(i) * n + j] * W2[size_t(j) * n + c];
            v[i] = t;
            g[i] = assoc_g(Mp + c, Mp, bz.points[i]);
            gv += g[i] * t;
            vv += t * t;
            gg += g[i] * g[i];
        }
        const double s = gv / vv;
        double rr = 0;
        for (int i = 0; i < n; ++i) rr += (s * v[i] - g[i]) * (s * v[i] - g[i]);
        if (!(std::sqrt(rr / gg) <= fit_tol)) continue;
        if (!(std::fabs(s) > 0) || !std::isfinite(s)) return "z eigenvector orthogonal to its Legendre function";
        resolved[c] = 1;
        for (int i = 0; i < n; ++i) {
            W2[size_t(i) * n + c] *= s;
            Wb2[size_t(c) * n + i] /= s;
        }
    }
    W.swap(W2);
    Wb.swap(Wb2);
    lre.swap(l2);
    return "";
}

// From the ordered z pencils of every M' block of one component (Wbz[iM],
// Wz[iM], n_z x n_z row-major; lz[iM] their eigenvalues; resolved[iM] the
// modes of order_and_scale_z), builds the joint z matrices Zj = [forward |
// backward], each (n_M n_z)^2 row-major over (slot, (iM, k)), and per slot
// the x and y pencil coefficients: A_x = -D_x + cx X_r2 S_x + V S_x,
// A_y = -D_y + cy Y_r2 S_y + Vhat S_y.  For each l the resolved modes
// (M', l - M') of consecutive M' form one chain of T_l; a mode that is not
// resolved is a slot of its own with its computed eigenvalue (cx = -lambda~,
// cy = J(J+1) - 2M'^2 - lambda~), as in the block-Jacobi variant.
std::string coupled_slots(const fm_problem *p, int nz, const std::vector<std::vector<double>> &Wbz,
                          const std::vector<std::vector<double>> &Wz, const std::vector<std::vector<double>> &lz,
                          const std::vector<std::vector<char>> &resolved, std::vector<double> &Zj,
                          std::vector<double> &cx, std::vector<double> &cy) {
    const int nM = p->nM, M0 = p->M0, J = p->desc.J;
    const int n = nM * nz;
    Zj.assign(size_t(2) * n * n, 0.0);
    cx.assign(n, 0.0);
    cy.assign(n, 0.0);
    double *Zf = Zj.data(), *Zb = Zj.data() + size_t(n) * n;
    int slot = 0;
    for (int l = M0; l <= J + nz - 1; ++l) {
        // the resolved modes of this l, cut into chains of consecutive M'
        std::vector<std::vector<int>> chains;
        for (int iM = 0; iM < nM; ++iM) {
            const int k = l - (M0 + iM);
            if (k < 0 || k >= nz || !resolved[iM][k]) continue;
            if (chains.empty() || chains.back().back() != iM - 1) chains.emplace_back();
            chains.back().push_back(iM);
        }
        for (const std::vector<int> &ms : chains) {
            const int nl = int(ms.size());
            std::vector<double> T(size_t(nl) * nl, 0.0), I(size_t(nl) * nl, 0.0);
            for (int q = 0; q < nl; ++q) {
                const int Mp = M0 + ms[q];
                I[size_t(q) * nl + q] = 1.0;
                T[size_t(q) * nl + q] = double(J) * (J + 1) - 2.0 * Mp * Mp + double(l) * (l + 1);
                if (q + 1 < nl) T[size_t(q) * nl + q + 1] = -lam_of(J, Mp) * std::sqrt(1.0 + (Mp == 0)) * lam_of(l, Mp);
                if (q >= 1) T[size_t(q) * nl + q - 1] = -lam_of(J, -Mp) * std::sqrt(1.0 + (Mp == 1)) * lam_of(l, -Mp);
            }
            std::vector<double> Ub, U, tre, tim;
            std::vector<signed char> ty;
            if (nl == 1) {      // a single M' for this l: nothing to diagonalise
                Ub = U = {1.0};
                tre = {T[0]};
            } else {
                std::string r = pencil_diag(nl, T, I, Ub, U, tre, tim, ty, nullptr);
                if (!r.empty()) return "M' coupling matrix: " + r;
                for (int q = 0; q < nl; ++q)
                    if (ty[q] != 0) return "M' coupling matrix has complex eigenvalues";
            }
            for (int m = 0; m < nl; ++m, ++slot) {
                cx[slot] = double(l) * (l + 1);
                cy[slot] = tre[m];
                for (int q = 0; q < nl; ++q) {
                    const int iM = ms[q], k = l - (M0 + iM);
                    const double uf = Ub[size_t(m) * nl + q], ub = U[size_t(q) * nl + m];
                    const double *wb = Wbz[iM].data() + size_t(k) * nz;   // row k of Wbar_z
                    for (int kk = 0; kk < nz; ++kk) Zf[size_t(slot) * n + iM * nz + kk] += uf * wb[kk];
                    for (int kk = 0; kk < nz; ++kk)                       // column k of W_z
                        Zb[size_t(iM * nz + kk) * n + slot] += Wz[iM][size_t(kk) * nz + k] * ub;
                }
            }
        }
    }
    // the modes that are not resolved, one slot each
    for (int iM = 0; iM < nM; ++iM)
        for (int k = 0; k < nz; ++k) {
            if (resolved[iM][k]) continue;
            const int Mp = M0 + iM;
            cx[slot] = -lz[iM][k];
            cy[slot] = double(J) * (J + 1) - 2.0 * Mp * Mp - lz[iM][k];
            const double *wb = Wbz[iM].data() + size_t(k) * nz;
            for (int kk = 0; kk < nz; ++kk) Zf[size_t(slot) * n + iM * nz + kk] = wb[kk];
            for (int kk = 0; kk < nz; ++kk) Zb[size_t(iM * nz + kk) * n + slot] = Wz[iM][size_t(kk) * nz + k];
            ++slot;
        }
    if (slot != n) return "slot count mismatch";
    return "";
}

}  // namespace fm

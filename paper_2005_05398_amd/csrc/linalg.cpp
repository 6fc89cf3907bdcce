// Host dense linear algebra for the preconditioner set-up (FP64).
//
// The operation D(A1, A2) of paper Sec. 3.2 (eq. (WW-scale)): matrices Wbar, W
// with Wbar A1 W = Lambda and Wbar A2 W = I.  With A2 = S nonsingular this is
// the eigendecomposition C W = W Lambda of C = S^-1 A1, and Wbar = (S W)^-1.
// The paper works in complex arithmetic; here complex-conjugate pairs a +- ib
// are kept as real 2x2 blocks [[a, b], [-b, a]] with the real and imaginary
// parts of the eigenvector as the two columns, so W, Wbar and Lambda stay real.
//
// Eigenvalues: balancing, Householder reduction to Hessenberg form, Francis
// implicit double-shift QR (Golub & Van Loan, Matrix Computations, Sec. 7.5).
// The balancing follows the published EISPACK routine BALANC (Parlett &
// Reinsch, Numer. Math. 13 (1969); powers-of-two row/column scaling until the
// norms settle), and the QR sweep the published EISPACK routine HQR (Martin,
// Peters & Wilkinson, Numer. Math. 14 (1970)): its search for two small
// consecutive subdiagonal elements and its exceptional shifts (0.75 s and
// -0.4375 s^2 on every tenth unsuccessful iteration) are kept.
// Eigenvectors: inverse iteration with the Hessenberg matrix (Sec. 7.6.1 there),
// mapped back through the Householder and balancing transforms.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "fm_internal.h"

namespace fm {

bool lu_factor(int n, std::vector<double> &a, std::vector<int> &piv) {
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::fabs(a[size_t(k) * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = std::fabs(a[size_t(i) * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return false;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(a[size_t(k) * n + j], a[size_t(p) * n + j]);
        double inv = 1.0 / a[size_t(k) * n + k];
        for (int i = k + 1; i < n; ++i) {
            double l = a[size_t(i) * n + k] * inv;
            a[size_t(i) * n + k] = l;
            if (l != 0.0)
                for (int j = k + 1; j < n; ++j) a[size_t(i) * n + j] -= l * a[size_t(k) * n + j];
        }
    }
    return true;
}

void lu_solve(int n, const std::vector<double> &lu, const std::vector<int> &piv, double *b) {
    for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= lu[size_t(i) * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= lu[size_t(i) * n + j] * b[j];
        b[i] = s / lu[size_t(i) * n + i];
    }
}

bool invert(int n, const std::vector<double> &a, std::vector<double> &inv) {
    std::vector<double> lu = a;
    std::vector<int> piv;
    if (!lu_factor(n, lu, piv)) return false;
    inv.assign(size_t(n) * n, 0.0);
    std::vector<double> col(n);
    for (int j = 0; j < n; ++j) {
        std::fill(col.begin(), col.end(), 0.0);
        col[j] = 1.0;
        lu_solve(n, lu, piv, col.data());
        for (int i = 0; i < n; ++i) inv[size_t(i) * n + j] = col[i];
    }
    return true;
}

namespace {

// Diagonal similarity by powers of two that evens out row and column norms;
// returns D with A <- D^-1 A D.
void balance(int n, std::vector<double> &a, std::vector<double> &d) {
    d.assign(n, 1.0);
    const double radix = 2.0, sq = radix * radix;
    bool done = false;
    for (int sweep = 0; sweep < 100 && !done; ++sweep) {
        done = true;
        for (int i = 0; i < n; ++i) {
            double c = 0, r = 0;
            for (int j = 0; j < n; ++j)
                if (j != i) {
                    c += std::fabs(a[size_t(j) * n + i]);
                    r += std::fabs(a[size_t(i) * n + j]);
                }
            if (c == 0.0 || r == 0.0) continue;
            double g = r / radix, f = 1.0, s = c + r;
            while (c < g) { f *= radix; c *= sq; }
            g = r * radix;
            while (c > g) { f /= radix; c /= sq; }
            if ((c + r) / f < 0.95 * s) {
                done = false;
                d[i] *= f;
                for (int j = 0; j < n; ++j) a[size_t(i) * n + j] /= f;
                for (int j = 0; j < n; ++j) a[size_t(j) * n + i] *= f;
            }
        }
    }
}

// Householder reduction to upper Hessenberg form: H = Q^T A Q.
void hessenberg(int n, std::vector<double> &a, std::vector<double> &Q) {
    Q.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Q[size_t(i) * n + i] = 1.0;
    std::vector<double> v(n), tmp(n);
    for (int k = 0; k + 2 < n; ++k) {
        double nrm = 0;
        for (int i = k + 1; i < n; ++i) nrm += a[size_t(i) * n + k] * a[size_t(i) * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        double x0 = a[size_t(k + 1) * n + k];
        double alpha = x0 >= 0 ? -nrm : nrm;
        std::fill(v.begin(), v.end(), 0.0);
        for (int i = k + 1; i < n; ++i) v[i] = a[size_t(i) * n + k];
        v[k + 1] -= alpha;
        double vn = 0;
        for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
        vn = std::sqrt(vn);
        if (vn == 0.0) continue;
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        // A <- (I - 2vv^T) A
        for (int j = 0; j < n; ++j) {
            double s = 0;
            for (int i = k + 1; i < n; ++i) s += v[i] * a[size_t(i) * n + j];
            for (int i = k + 1; i < n; ++i) a[size_t(i) * n + j] -= 2 * v[i] * s;
        }
        // A <- A (I - 2vv^T),  Q <- Q (I - 2vv^T)
        for (int i = 0; i < n; ++i) {
            double s = 0, sq = 0;
            for (int j = k + 1; j < n; ++j) {
                s += a[size_t(i) * n + j] * v[j];
                sq += Q[size_t(i) * n + j] * v[j];
            }
            for (int j = k + 1; j < n; ++j) {
                a[size_t(i) * n + j] -= 2 * s * v[j];
                Q[size_t(i) * n + j] -= 2 * sq * v[j];
            }
        }
        for (int i = k + 2; i < n; ++i) a[size_t(i) * n + k] = 0.0;
    }
}

// Eigenvalues of an upper Hessenberg matrix by the Francis implicit
// double-shift QR iteration with deflation (matrix destroyed).
bool hessenberg_eigenvalues(int n, std::vector<double> a, std::vector<double> &wr, std::vector<double> &wi) {
    auto A = [&](int i, int j) -> double & { return a[size_t(i) * n + j]; };
    wr.assign(n, 0.0);
    wi.assign(n, 0.0);
    double anorm = 0;
    for (int i = 0; i < n; ++i)
        for (int j = std::max(i - 1, 0); j < n; ++j) anorm += std::fabs(A(i, j));
    int hi = n - 1;
    double shift_acc = 0.0;
    while (hi >= 0) {
        int its = 0, lo;
        for (;;) {
            // deflation: find the bottom of the unreduced block ending at hi
            for (lo = hi; lo >= 1; --lo) {
                double s = std::fabs(A(lo - 1, lo - 1)) + std::fabs(A(lo, lo));
                if (s == 0.0) s = anorm;
                if (std::fabs(A(lo, lo - 1)) + s == s) {
                    A(lo, lo - 1) = 0.0;
                    break;
                }
            }
            double x = A(hi, hi);
            if (lo == hi) {                       // 1x1 block converged
                wr[hi] = x + shift_acc;
                wi[hi] = 0.0;
                hi -= 1;
                break;
            }
            double y = A(hi - 1, hi - 1), w = A(hi, hi - 1) * A(hi - 1, hi);
            if (lo == hi - 1) {                   // 2x2 block converged
                double p = 0.5 * (y - x), q = p * p + w, z = std::sqrt(std::fabs(q));
                x += shift_acc;
                if (q >= 0.0) {
                    z = p + std::copysign(z, p);
                    wr[hi - 1] = wr[hi] = x + z;
                    if (z != 0.0) wr[hi] = x - w / z;
                    wi[hi - 1] = wi[hi] = 0.0;
                } else {
                    wr[hi - 1] = wr[hi] = x + p;
                    wi[hi - 1] = z;
                    wi[hi] = -z;
                }
                hi -= 2;
                break;
            }
            if (its >= 80) return false;
            if (its > 0 && its % 10 == 0) {       // exceptional shift
                shift_acc += x;
                for (int i = 0; i <= hi; ++i) A(i, i) -= x;
                double s = std::fabs(A(hi, hi - 1)) + std::fabs(A(hi - 1, hi - 2));
                x = y = 0.75 * s;
                w = -0.4375 * s * s;
            }
            ++its;
            // look for two consecutive small sub-diagonal elements
            int m;
            double p = 0, q = 0, r = 0, z;
            for (m = hi - 2; m >= lo; --m) {
                z = A(m, m);
                double rr = x - z, ss = y - z;
                p = (rr * ss - w) / A(m + 1, m) + A(m, m + 1);
                q = A(m + 1, m + 1) - z - rr - ss;
                r = A(m + 2, m + 1);
                double sc = std::fabs(p) + std::fabs(q) + std::fabs(r);
                p /= sc; q /= sc; r /= sc;
                if (m == lo) break;
                double u = std::fabs(A(m, m - 1)) * (std::fabs(q) + std::fabs(r));
                double v = std::fabs(p) * (std::fabs(A(m - 1, m - 1)) + std::fabs(z) + std::fabs(A(m + 1, m + 1)));
                if (u + v == v) break;
            }
            for (int i = m + 2; i <= hi; ++i) {
                A(i, i - 2) = 0.0;
                if (i != m + 2) A(i, i - 3) = 0.0;
            }
            // double-shift QR sweep on rows/columns m..hi (bulge chase)
            for (int k = m; k <= hi - 1; ++k) {
                if (k != m) {
                    p = A(k, k - 1);
                    q = A(k + 1, k - 1);
                    r = (k != hi - 1) ? A(k + 2, k - 1) : 0.0;
                    x = std::fabs(p) + std::fabs(q) + std::fabs(r);
                    if (x != 0.0) { p /= x; q /= x; r /= x; }
                }
                double s = std::copysign(std::sqrt(p * p + q * q + r * r), p);
                if (s == 0.0) continue;
                if (k == m) {
                    if (lo != m) A(k, k - 1) = -A(k, k - 1);
                } else {
                    A(k, k - 1) = -s * x;
                }
                p += s;
                x = p / s;
                y = q / s;
                z = r / s;
                q /= p;
                r /= p;
                for (int j = k; j <= hi; ++j) {           // rows k..k+2
                    double t = A(k, j) + q * A(k + 1, j);
                    if (k != hi - 1) {
                        t += r * A(k + 2, j);
                        A(k + 2, j) -= t * z;
                    }
                    A(k + 1, j) -= t * y;
                    A(k, j) -= t * x;
                }
                int imax = std::min(hi, k + 3);
                for (int i = lo; i <= imax; ++i) {         // columns k..k+2
                    double t = x * A(i, k) + y * A(i, k + 1);
                    if (k != hi - 1) {
                        t += z * A(i, k + 2);
                        A(i, k + 2) -= t * r;
                    }
                    A(i, k + 1) -= t * q;
                    A(i, k) -= t;
                }
            }
        }
    }
    return true;
}

using cplx = std::complex<double>;

// Null vector of (H - lambda I), H upper Hessenberg, by two steps of inverse
// iteration with a Hessenberg LU (row interchanges between neighbours).
std::vector<cplx> inverse_iteration(int n, const std::vector<double> &H, cplx lambda, double hnorm) {
    std::vector<cplx> U(size_t(n) * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) U[size_t(i) * n + j] = H[size_t(i) * n + j] - (i == j ? lambda : 0.0);
    std::vector<cplx> mult(n, 0.0);
    std::vector<char> swapped(n, 0);
    const double tiny = 1e-15 * std::max(hnorm, 1e-300);
    for (int k = 0; k + 1 < n; ++k) {
        cplx &pk = U[size_t(k) * n + k];
        cplx &sk = U[size_t(k + 1) * n + k];
        if (std::abs(sk) > std::abs(pk)) {
            for (int j = k; j < n; ++j) std::swap(U[size_t(k) * n + j], U[size_t(k + 1) * n + j]);
            swapped[k] = 1;
        }
        cplx piv = U[size_t(k) * n + k];
        if (std::abs(piv) < tiny) piv = U[size_t(k) * n + k] = tiny;
        cplx l = U[size_t(k + 1) * n + k] / piv;
        mult[k] = l;
        U[size_t(k + 1) * n + k] = 0.0;
        for (int j = k + 1; j < n; ++j) U[size_t(k + 1) * n + j] -= l * U[size_t(k) * n + j];
    }
    if (std::abs(U[size_t(n - 1) * n + n - 1]) < tiny) U[size_t(n - 1) * n + n - 1] = tiny;
    auto solve = [&](std::vector<cplx> &b) {
        for (int k = 0; k + 1 < n; ++k) {
            if (swapped[k]) std::swap(b[k], b[k + 1]);
            b[k + 1] -= mult[k] * b[k];
        }
        for (int i = n - 1; i >= 0; --i) {
            cplx s = b[i];
            for (int j = i + 1; j < n; ++j) s -= U[size_t(i) * n + j] * b[j];
            b[i] = s / U[size_t(i) * n + i];
        }
        double nrm = 0;
        for (auto &v : b) nrm += std::norm(v);
        nrm = std::sqrt(nrm);
        for (auto &v : b) v /= nrm;
    };
    std::vector<cplx> b(n);
    for (int i = 0; i < n; ++i) b[i] = 1.0 + 0.1 * std::sin(1.0 + 7.3 * i);   // fixed start vector
    solve(b);
    solve(b);
    return b;
}


// Fallback for a value whose Hessenberg-form vector misses the residual test
// (a tight cluster, or a balancing with a wide range): inverse iteration on the
// original matrix A with a full LU (partial pivoting), from a start vector
// orthogonalised against the vectors already accepted, up to six steps, each
// checked on ||A v - lambda v||.  Returns the residual reached.
double inverse_iteration_full(int n, const std::vector<double> &A, cplx lambda, double tol,
                              const std::vector<std::vector<cplx>> &prev, std::vector<cplx> &v) {
    std::vector<cplx> U(size_t(n) * n);
    double anorm = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            U[size_t(i) * n + j] = A[size_t(i) * n + j] - (i == j ? lambda : 0.0);
            anorm = std::max(anorm, std::fabs(A[size_t(i) * n + j]));
        }
    const double tiny = 1e-15 * std::max(anorm, 1e-300);
    std::vector<int> piv(n);
    for (int k = 0; k < n; ++k) {
        int pr = k;
        for (int i = k + 1; i < n; ++i)
            if (std::abs(U[size_t(i) * n + k]) > std::abs(U[size_t(pr) * n + k])) pr = i;
        piv[k] = pr;
        if (pr != k)
            for (int j = 0; j < n; ++j) std::swap(U[size_t(k) * n + j], U[size_t(pr) * n + j]);
        if (std::abs(U[size_t(k) * n + k]) < tiny) U[size_t(k) * n + k] = tiny;
        for (int i = k + 1; i < n; ++i) {
            const cplx l = U[size_t(i) * n + k] / U[size_t(k) * n + k];
            U[size_t(i) * n + k] = l;
            for (int j = k + 1; j < n; ++j) U[size_t(i) * n + j] -= l * U[size_t(k) * n + j];
        }
    }
    auto normalise = [&](std::vector<cplx> &b) {
        double nrm = 0;
        for (auto &t : b) nrm += std::norm(t);
        nrm = std::sqrt(nrm);
        for (auto &t : b) t /= nrm;
    };
    v.assign(n, 0.0);
    for (int i = 0; i < n; ++i) v[i] = cplx(1.0 + 0.3 * std::sin(2.0 + 5.1 * i), 0.2 * std::cos(1.0 + 3.7 * i));
    for (const auto &u : prev) {                       // away from the vectors already found
        cplx d = 0.0;
        for (int i = 0; i < n; ++i) d += std::conj(u[i]) * v[i];
        for (int i = 0; i < n; ++i) v[i] -= d * u[i];
    }
    normalise(v);
    double res = 1e300;
    for (int it = 0; it < 6 && !(res <= tol); ++it) {
        for (int k = 0; k < n; ++k) std::swap(v[k], v[piv[k]]);
        for (int i = 1; i < n; ++i)
            for (int j = 0; j < i; ++j) v[i] -= U[size_t(i) * n + j] * v[j];
        for (int i = n - 1; i >= 0; --i) {
            cplx t = v[i];
            for (int j = i + 1; j < n; ++j) t -= U[size_t(i) * n + j] * v[j];
            v[i] = t / U[size_t(i) * n + i];
        }
        normalise(v);
        res = 0;
        for (int i = 0; i < n; ++i) {
            cplx t = -lambda * v[i];
            for (int j = 0; j < n; ++j) t += A[size_t(i) * n + j] * v[j];
            res = std::max(res, std::abs(t));
        }
    }
    return res;
}

}  // namespace

std::string pencil_diag(int n, const std::vector<double> &A1, const std::vector<double> &A2,
                        std::vector<double> &Wbar, std::vector<double> &W, std::vector<double> &lre,
                        std::vector<double> &lim, std::vector<signed char> &type, double *err) {
    // C = A2^-1 A1
    std::vector<double> lu = A2;
    std::vector<int> piv;
    if (!lu_factor(n, lu, piv)) return "singular collocation matrix";
    std::vector<double> C(size_t(n) * n);
    std::vector<double> col(n);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) col[i] = A1[size_t(i) * n + j];
        lu_solve(n, lu, piv, col.data());
        for (int i = 0; i < n; ++i) C[size_t(i) * n + j] = col[i];
    }
    std::vector<double> D;
    balance(n, C, D);
    std::vector<double> Q;
    hessenberg(n, C, Q);
    double hnorm = 0;
    for (double v : C) hnorm = std::max(hnorm, std::fabs(v));
    std::vector<double> wr, wi;
    if (!hessenberg_eigenvalues(n, C, wr, wi)) return "QR iteration did not converge";
    // order: increasing real part; a complex pair as (a + ib, a - ib), b > 0
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) {
        if (wr[i] != wr[j]) return wr[i] < wr[j];
        return wi[i] > wi[j];
    });
    W.assign(size_t(n) * n, 0.0);
    lre.assign(n, 0.0);
    lim.assign(n, 0.0);
    type.assign(n, 0);
    for (int c = 0; c < n; ++c) {
        int e = ord[c];
        cplx lam(wr[e], wi[e]);
        bool pair = wi[e] != 0.0;
        if (pair && !(wi[e] > 0.0 && c + 1 < n && wi[ord[c + 1]] == -wi[e])) return "unpaired complex eigenvalue";
        std::vector<cplx> y = inverse_iteration(n, C, lam, hnorm);
        // v = D (Q y)
        std::vector<cplx> v(n, 0.0);
        for (int i = 0; i < n; ++i) {
            cplx s = 0.0;
            for (int j = 0; j < n; ++j) s += Q[size_t(i) * n + j] * y[j];
            v[i] = s * D[i];
        }
        double nrm = 0;
        for (auto &t : v) nrm += std::norm(t);
        nrm = std::sqrt(nrm);
        if (!pair) {
            for (int i = 0; i < n; ++i) W[size_t(i) * n + c] = v[i].real() / nrm;
            lre[c] = lam.real();
        } else {
            for (int i = 0; i < n; ++i) {
                W[size_t(i) * n + c] = v[i].real() / nrm;
                W[size_t(i) * n + c + 1] = v[i].imag() / nrm;
            }
            lre[c] = lre[c + 1] = lam.real();
            lim[c] = lam.imag();
            lim[c + 1] = -lam.imag();
            type[c] = 1;
            type[c + 1] = 2;
            ++c;
        }
    }
    // Wbar = (A2 W)^-1
    std::vector<double> SW(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            double a = A2[size_t(i) * n + k];
            if (a == 0.0) continue;
            for (int j = 0; j < n; ++j) SW[size_t(i) * n + j] += a * W[size_t(k) * n + j];
        }
    if (!invert(n, SW, Wbar)) return "eigenvector matrix is singular";
    // accuracy check: Wbar A1 W = Lambda, Wbar A2 W = I
    double e1 = 0, e2 = 0, lmax = 0;
    std::vector<double> T(size_t(n) * n, 0.0), U(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            double a1 = A1[size_t(i) * n + k], a2 = A2[size_t(i) * n + k];
            for (int j = 0; j < n; ++j) {
                double w = W[size_t(k) * n + j];
                T[size_t(i) * n + j] += a1 * w;
                U[size_t(i) * n + j] += a2 * w;
            }
        }
    for (int c = 0; c < n; ++c) lmax = std::max(lmax, std::hypot(lre[c], lim[c]));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s1 = 0, s2 = 0;
            for (int k = 0; k < n; ++k) {
                double wb = Wbar[size_t(i) * n + k];
                s1 += wb * T[size_t(k) * n + j];
                s2 += wb * U[size_t(k) * n + j];
            }
            double want1 = 0;
            if (i == j) want1 = lre[i];
            else if (j == i + 1 && type[i] == 1) want1 = lim[i];
            else if (j == i - 1 && type[i] == 2) want1 = lim[i];
            e1 = std::max(e1, std::fabs(s1 - want1));
            e2 = std::max(e2, std::fabs(s2 - (i == j ? 1.0 : 0.0)));
        }
    double e = std::max(e1 / std::max(lmax, 1e-300), e2);
    if (err) *err = e;
    if (!(e < 1e-6)) return "generalized eigendecomposition failed its accuracy check";
    return "";
}

std::string dense_eig_by_modulus(int n, const std::vector<double> &A, int nmin, int ncols, std::vector<double> &wr,
                                 std::vector<double> &wi, std::vector<double> &V, std::vector<signed char> &type,
                                 int &nv) {
    std::vector<double> C = A, D, Q;
    balance(n, C, D);
    hessenberg(n, C, Q);
    double hnorm = 0;
    for (double v : C) hnorm = std::max(hnorm, std::fabs(v));
    std::vector<double> r, im;
    if (!hessenberg_eigenvalues(n, C, r, im)) return "QR iteration did not converge";
    // decreasing modulus; a complex pair as (a + ib, a - ib), b > 0
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) {
        const double mi = std::hypot(r[i], im[i]), mj = std::hypot(r[j], im[j]);
        if (mi != mj) return mi > mj;
        return im[i] > im[j];
    });
    wr.assign(n, 0.0);
    wi.assign(n, 0.0);
    for (int c = 0; c < n; ++c) {
        wr[c] = r[ord[c]];
        wi[c] = im[ord[c]];
    }
    for (int c = 0; c + 1 < n; ++c)       // pairs must sit together (equal modulus)
        if (wi[c] > 0.0 && !(wi[c + 1] == -wi[c] && wr[c + 1] == wr[c])) return "unpaired complex eigenvalue";
    // eigenvectors of the leading values (at least ncols columns, pairs whole)
    std::vector<std::vector<double>> cols;
    std::vector<std::vector<cplx>> found;             // accepted vectors (unit, complex)
    type.clear();
    double anorm = 0;
    for (double v : A) anorm = std::max(anorm, std::fabs(v));
    for (int c = 0; c < n && (int)cols.size() < ncols; ++c) {
        const cplx lam(wr[c], wi[c]);
        std::vector<cplx> y = inverse_iteration(n, C, lam, hnorm);
        std::vector<cplx> v(n, 0.0);
        for (int i = 0; i < n; ++i) {
            cplx t = 0.0;
            for (int j = 0; j < n; ++j) t += Q[size_t(i) * n + j] * y[j];
            v[i] = t * D[i];
        }
        double nrm = 0;
        for (auto &t : v) nrm += std::norm(t);
        nrm = std::sqrt(nrm);
        for (auto &t : v) t /= nrm;
        // residual of the original matrix
        double res = 0;
        for (int i = 0; i < n; ++i) {
            cplx t = -lam * v[i];
            for (int j = 0; j < n; ++j) t += A[size_t(i) * n + j] * v[j];
            res = std::max(res, std::abs(t));
        }
        const double tol = 1e-11 * std::max(anorm, std::abs(lam));
        if (!(res <= tol)) res = inverse_iteration_full(n, A, lam, tol, found, v);
        if (!(res <= tol)) {
            if ((int)cols.size() < nmin) return "inverse iteration did not converge";
            break;                                    // keep the vectors found so far
        }
        found.push_back(v);
        std::vector<double> re(n), ii(n);
        for (int i = 0; i < n; ++i) {
            re[i] = v[i].real();
            ii[i] = v[i].imag();
        }
        cols.push_back(re);
        if (wi[c] != 0.0) {
            cols.push_back(ii);
            type.push_back(1);
            type.push_back(2);
            ++c;                                      // the conjugate shares the pair's columns
        } else {
            type.push_back(0);
        }
    }
    nv = int(cols.size());
    V.assign(size_t(n) * nv, 0.0);
    for (int c = 0; c < nv; ++c)
        for (int i = 0; i < n; ++i) V[size_t(i) * nv + c] = cols[c][i];
    return "";
}

}  // namespace fm

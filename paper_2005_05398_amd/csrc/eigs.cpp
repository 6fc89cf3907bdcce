// Bound-state energies by shift-invert Arnoldi (Sec. 3.1, eq. (FM-lin): the
// energies are eigenvalues of H c = E S c, and the method iterates with the
// inverse of H - E* S; Sec. 4 uses implicitly restarted Arnoldi for it).
//
// T = (H - sigma S)^-1 S has the eigenvalues theta = 1/(E - sigma), so the
// energies nearest sigma are T's eigenvalues of largest modulus.  Each Arnoldi
// step applies S on the device and solves with H - sigma S by the library's
// flexible GMRES; the basis vectors live on the device and are orthogonalised
// twice by classical Gram-Schmidt.  Restarts follow Krylov-Schur (Stewart,
// SIAM J. Matrix Anal. Appl. 23 (2001)): with A V_m = V_m H_m + beta v_{m+1} e_m^T,
// an orthonormal basis Q of the invariant subspace of H_m spanned by the kept
// Ritz vectors gives A (V_m Q) = (V_m Q)(Q^T H_m Q) + v_{m+1} (beta e_m^T Q),
// which is the relation the next expansion continues from; this is
// mathematically the same restart as the implicit shifts of IRAM.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "fm_problem.h"

namespace fm {

namespace {

fm_status efail(fm_status s, const std::string &m) {
    set_error(m);
    return s;
}

#define EIG_HIP(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return efail(FM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DevMem {
    std::vector<void *> ptrs;
    ~DevMem() {
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        for (void *q : ptrs) (void)hipFree(q);
    }
    bool get(double **out, size_t n) {
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        void *q = nullptr;
        if (hipMalloc(&q, sizeof(double) * std::max<size_t>(n, 1)) != hipSuccess) return false;
        ptrs.push_back(q);
        *out = static_cast<double *>(q);
        return true;
    }
};

// One Ritz value (a real one, or the first of a complex pair) of the m x m
// projected matrix: its columns in W (col, and col + 1 for a pair).
struct Ritz {
    int col;
    bool pair;
    double re, im, mag;
};

}  // namespace

}  // namespace fm

using namespace fm;

extern "C" fm_status fm_eigs(fm_problem *p, double sigma, const fm_eigs_opts *o, const double *v0_dev, double *E_re,
                             double *E_im, double *resid, double *vec_dev, fm_eigs_info *info, void *stream) {
    if (!p || !o || !E_re || !E_im || !resid) return efail(FM_E_INVALID, "bad argument");
    const int nev = o->nev, ncv = o->ncv;
    const long long N = p->N;
    if (nev < 1 || ncv < nev + 2 || ncv > 256 || ncv > N) return efail(FM_E_INVALID, "need 1 <= nev, nev + 2 <= ncv <= min(256, N)");
    if (!(o->tol > 0) || o->max_restarts < 1 || !std::isfinite(sigma)) return efail(FM_E_INVALID, "bad tol, max_restarts or sigma");
    const fm_solve_opts &in = o->inner;
    if (in.restart < 1 || in.restart > MAX_RESTART || !(in.rtol > 0) || in.max_iters < 1 ||
        (in.prec != FM_FP64 && in.prec != FM_FP32 && in.prec != FM_BF16X3))
        return efail(FM_E_INVALID, "bad inner solve options");
    Busy busy(p);
    if (!busy.ok) return efail(FM_E_BUSY, "problem handle in use");
    EIG_HIP(hipSetDevice(p->desc.device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    fm_solve_opts inner = in;
    inner.x0_is_guess = 0;

    DevMem mem;
    double *V, *tmp, *sv, *part, *dsmall;
    const int nblk = cols_dot_blocks(N);
    if (!mem.get(&V, size_t(ncv + 1) * N) || !mem.get(&tmp, size_t(ncv) * N) || !mem.get(&sv, N) ||
        !mem.get(&part, size_t(nblk) * (ncv + 1)) || !mem.get(&dsmall, size_t(ncv) * ncv + ncv + 1))
        return efail(FM_E_NOMEM, "eigensolver workspace allocation failed");
    std::vector<double> h(ncv + 1), h2(ncv + 1);
    auto dots = [&](int ncol, const double *w, std::vector<double> &out) -> fm_status {
        launch_cols_dot(V, ncol, w, N, part, dsmall, st);
        EIG_HIP(hipGetLastError());
        EIG_HIP(hipMemcpyAsync(out.data(), dsmall, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
        EIG_HIP(hipStreamSynchronize(st));
        return FM_OK;
    };
    auto norm_of = [&](const double *w, double &nrm) -> fm_status {
        launch_cols_dot(w, 1, w, N, part, dsmall, st);
        EIG_HIP(hipGetLastError());
        double v = 0;
        EIG_HIP(hipMemcpyAsync(&v, dsmall, sizeof(double), hipMemcpyDeviceToHost, st));
        EIG_HIP(hipStreamSynchronize(st));
        nrm = std::sqrt(std::max(v, 0.0));
        return FM_OK;
    };
    auto put_small = [&](const double *src, int n) -> fm_status {
        EIG_HIP(hipMemcpyAsync(dsmall, src, sizeof(double) * n, hipMemcpyHostToDevice, st));
        EIG_HIP(hipStreamSynchronize(st));
        return FM_OK;
    };

    // start vector
    if (v0_dev) launch_copy(V, v0_dev, N, st);
    else launch_fill(V, N, 1.0, st);
    double nrm = 0;
    fm_status r = norm_of(V, nrm);
    if (r != FM_OK) return r;
    if (!(nrm > 0) || !std::isfinite(nrm)) return efail(FM_E_INVALID, "start vector is zero or not finite");
    launch_scale_vec(V, 1.0 / nrm, N, st);

    std::vector<double> H(size_t(ncv + 1) * ncv, 0.0);   // row-major (ncv + 1) x ncv
    auto Hat = [&](int i, int j) -> double & { return H[size_t(i) * ncv + j]; };
    fm_eigs_info inf{};
    int k = 0;                 // columns kept by the last restart
    std::vector<Ritz> ritz;
    std::vector<double> Wr;    // Ritz vectors of the projected matrix (m x nvr, row-major)
    int nvr = 0;
    int m = ncv;
    double beta = 0;
    bool exact = false;        // the Krylov space became invariant
    // Ritz residual estimate |beta| |last component of y| (||y|| = 1)
    auto est = [&](const Ritz &z) {
        const double v = Wr[size_t(m - 1) * nvr + z.col];
        const double u = z.pair ? Wr[size_t(m - 1) * nvr + z.col + 1] : 0.0;
        return std::fabs(beta) * std::hypot(v, u);
    };
    for (int rs = 0;; ++rs) {
        // expand to m = ncv columns
        m = ncv;
        for (int j = k; j < ncv; ++j) {
            const double *vj = V + size_t(j) * N;
            double *w = V + size_t(j + 1) * N;
            launch_mass(p->pd, 1, vj, sv, st);
            EIG_HIP(hipGetLastError());
            fm_solve_result res{};
            r = solve_locked(p, 1, &sigma, sv, w, &inner, &res, st);
            if (r == FM_E_NONFINITE) return efail(FM_E_NONFINITE, "inner solve produced non-finite values");
            if (r != FM_OK && r != FM_E_NOT_CONVERGED) return r;
            ++inf.solves;
            inf.inner_iters += res.iters;
            if (res.status != FM_OK) ++inf.inner_failures;
            double w0 = 0;
            r = norm_of(w, w0);
            if (r != FM_OK) return r;
            // classical Gram-Schmidt, twice
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<double> &hh = pass == 0 ? h : h2;
                r = dots(j + 1, w, hh);
                if (r != FM_OK) return r;
                r = put_small(hh.data(), j + 1);
                if (r != FM_OK) return r;
                launch_cols_axpy(w, V, j + 1, dsmall, N, st);
                EIG_HIP(hipGetLastError());
            }
            for (int i = 0; i <= j; ++i) Hat(i, j) += h[i] + h2[i];
            r = norm_of(w, beta);
            if (r != FM_OK) return r;
            if (!std::isfinite(beta)) return efail(FM_E_NONFINITE, "non-finite Arnoldi vector");
            Hat(j + 1, j) = beta;
            if (beta <= 1e-13 * std::max(w0, 1e-300)) {    // invariant subspace: Ritz values exact
                m = j + 1;
                exact = true;
                beta = 0;
                break;
            }
            launch_scale_vec(w, 1.0 / beta, N, st);
        }
        // Ritz values of the m x m projected matrix by decreasing modulus, and
        // vectors of the leading ones (enough for the wanted and the kept values)
        std::vector<double> Hm(size_t(m) * m), wr, wi;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Hm[size_t(i) * m + j] = Hat(i, j);
        const int target = nev + (ncv - nev) / 2;
        std::vector<signed char> vty;
        std::string e = dense_eig_by_modulus(m, Hm, std::min(m, nev + 1), std::min(m, std::max(nev, target) + 1), wr,
                                             wi, Wr, vty, nvr);
        if (!e.empty()) return efail(FM_E_NOT_CONVERGED, "projected eigenproblem: " + e);
        ritz.clear();
        for (int c = 0, v = 0; c < nvr; ++v) {
            const bool pair = vty[c] == 1;
            ritz.push_back(Ritz{c, pair, wr[v], pair ? wi[v] : 0.0, std::hypot(wr[v], pair ? wi[v] : 0.0)});
            c += pair ? 2 : 1;
            if (pair) ++v;
        }
        // converged count in eigenvalues (a pair counts twice, up to nev)
        int nconv = 0, counted = 0;
        for (const Ritz &z : ritz) {
            if (counted >= nev) break;
            const int take = std::min(z.pair ? 2 : 1, nev - counted);
            if (est(z) <= o->tol * z.mag) nconv += take;
            counted += take;
        }
        inf.nconv = nconv;
        inf.restarts = rs;
        const bool done = exact || nconv >= std::min(nev, counted) || rs >= o->max_restarts;
        if (done) break;
        // restart: keep the Ritz vectors of the largest values (pairs whole)
        int keep_cols = 0;
        std::vector<int> cols;
        for (const Ritz &z : ritz) {
            const int add = z.pair ? 2 : 1;
            if (keep_cols + add > std::min(target, ncv - 1)) break;
            cols.push_back(z.col);
            if (z.pair) cols.push_back(z.col + 1);
            keep_cols += add;
        }
        if (keep_cols < 1) return efail(FM_E_NOT_CONVERGED, "restart kept no Ritz vector");
        // orthonormal basis Q (m x keep) of the kept Ritz vectors: modified Gram-Schmidt, twice
        const int kp = keep_cols;
        std::vector<double> Q(size_t(m) * kp);
        for (int c = 0; c < kp; ++c)
            for (int i = 0; i < m; ++i) Q[size_t(i) * kp + c] = Wr[size_t(i) * nvr + cols[c]];
        for (int c = 0; c < kp; ++c) {
            for (int pass = 0; pass < 2; ++pass)
                for (int d = 0; d < c; ++d) {
                    double s = 0;
                    for (int i = 0; i < m; ++i) s += Q[size_t(i) * kp + d] * Q[size_t(i) * kp + c];
                    for (int i = 0; i < m; ++i) Q[size_t(i) * kp + c] -= s * Q[size_t(i) * kp + d];
                }
            double s = 0;
            for (int i = 0; i < m; ++i) s += Q[size_t(i) * kp + c] * Q[size_t(i) * kp + c];
            s = std::sqrt(s);
            if (!(s > 1e-10)) return efail(FM_E_NOT_CONVERGED, "kept Ritz vectors are linearly dependent");
            for (int i = 0; i < m; ++i) Q[size_t(i) * kp + c] /= s;
        }
        // G = Q^T H_m Q, b = beta e_m^T Q
        std::vector<double> HQ(size_t(m) * kp, 0.0), G(size_t(kp) * kp, 0.0);
        for (int i = 0; i < m; ++i)
            for (int l = 0; l < m; ++l) {
                const double a = Hm[size_t(i) * m + l];
                if (a == 0.0) continue;
                for (int c = 0; c < kp; ++c) HQ[size_t(i) * kp + c] += a * Q[size_t(l) * kp + c];
            }
        for (int a = 0; a < kp; ++a)
            for (int c = 0; c < kp; ++c) {
                double s = 0;
                for (int i = 0; i < m; ++i) s += Q[size_t(i) * kp + a] * HQ[size_t(i) * kp + c];
                G[size_t(a) * kp + c] = s;
            }
        // device: V[0:kp] = V[0:m] Q, V[kp] = V[m]
        r = put_small(Q.data(), m * kp);
        if (r != FM_OK) return r;
        launch_cols_combine(V, m, dsmall, kp, tmp, N, st);
        launch_copy(V, tmp, size_t(kp) * N, st);
        launch_copy(V + size_t(kp) * N, V + size_t(m) * N, N, st);
        EIG_HIP(hipGetLastError());
        std::fill(H.begin(), H.end(), 0.0);
        for (int a = 0; a < kp; ++a)
            for (int c = 0; c < kp; ++c) Hat(a, c) = G[size_t(a) * kp + c];
        for (int c = 0; c < kp; ++c) Hat(kp, c) = beta * Q[size_t(m - 1) * kp + c];
        k = kp;
    }
    // results: nev values nearest sigma (a pair gives E and its conjugate)
    int slot = 0;
    std::vector<double> Y;
    std::vector<int> vslots;
    for (const Ritz &z : ritz) {
        for (int part_i = 0; part_i < (z.pair ? 2 : 1) && slot < nev; ++part_i, ++slot) {
            const double th_re = z.re, th_im = part_i == 0 ? z.im : -z.im;
            const double mag2 = z.mag * z.mag;
            E_re[slot] = sigma + th_re / mag2;
            E_im[slot] = -th_im / mag2;
            resid[slot] = est(z) / std::max(z.mag, 1e-300);
            if (vec_dev) {
                // slot gets the real part (first of a pair: then the imaginary part in the next slot)
                const int col = z.col + part_i;
                for (int i = 0; i < m; ++i) Y.push_back(Wr[size_t(i) * nvr + col]);
                vslots.push_back(slot);
            }
        }
        if (slot >= nev) break;
    }
    for (; slot < nev; ++slot) {                      // fewer Ritz values than nev (tiny problems)
        E_re[slot] = E_im[slot] = std::nan("");
        resid[slot] = std::nan("");
    }
    if (vec_dev && !vslots.empty()) {
        const int nv = int(vslots.size());
        std::vector<double> Yt(size_t(m) * nv);          // row-major m x nv
        for (int c = 0; c < nv; ++c)
            for (int i = 0; i < m; ++i) Yt[size_t(i) * nv + c] = Y[size_t(c) * m + i];
        r = put_small(Yt.data(), m * nv);
        if (r != FM_OK) return r;
        launch_cols_combine(V, m, dsmall, nv, tmp, N, st);
        for (int c = 0; c < nv; ++c) launch_copy(vec_dev + size_t(vslots[c]) * N, tmp + size_t(c) * N, N, st);
        EIG_HIP(hipGetLastError());
    }
    EIG_HIP(hipStreamSynchronize(st));
    if (info) *info = inf;
    if (inf.nconv < nev) return efail(FM_E_NOT_CONVERGED, "not every wanted Ritz pair met tol");
    return FM_OK;
}

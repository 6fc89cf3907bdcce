// Host-only inspection entry points (include/fm_host.h).
#include <cstring>

#include "../../include/fm_host.h"
#include "fm_problem.h"

using namespace fm;

extern "C" {

fm_status fm_host_basis(const fm_dim *dim, int is_z, double *points, double *S, double *D1, double *D2) {
    if (!dim) {
        set_error("null argument");
        return FM_E_INVALID;
    }
    Basis1D b;
    std::string e = b.init(*dim, is_z != 0);
    if (!e.empty()) {
        set_error(e);
        return FM_E_INVALID;
    }
    if (points) std::memcpy(points, b.points.data(), sizeof(double) * b.n);
    double *outs[3] = {S, D1, D2};
    for (int k = 0; k < 3; ++k)
        if (outs[k]) {
            std::vector<double> M = b.dense(k);
            std::memcpy(outs[k], M.data(), sizeof(double) * M.size());
        }
    return FM_OK;
}

fm_status fm_host_pencil(int n, const double *A1, const double *A2, double *Wbar, double *W, double *lre,
                         double *lim, signed char *type, double *err) {
    if (n < 1 || !A1 || !A2) {
        set_error("bad argument");
        return FM_E_INVALID;
    }
    std::vector<double> a1(A1, A1 + size_t(n) * n), a2(A2, A2 + size_t(n) * n), wb, w, lr, li;
    std::vector<signed char> ty;
    double e = 0;
    std::string r = pencil_diag(n, a1, a2, wb, w, lr, li, ty, &e);
    if (err) *err = e;
    if (!r.empty()) {
        set_error(r);
        return FM_E_PENCIL;
    }
    if (Wbar) std::memcpy(Wbar, wb.data(), sizeof(double) * wb.size());
    if (W) std::memcpy(W, w.data(), sizeof(double) * w.size());
    if (lre) std::memcpy(lre, lr.data(), sizeof(double) * n);
    if (lim) std::memcpy(lim, li.data(), sizeof(double) * n);
    if (type) std::memcpy(type, ty.data(), n);
    return FM_OK;
}

fm_status fm_host_setup_check(const fm_problem_desc *desc, double *max_err, int *complex_pairs, size_t *n_unknowns) {
    if (!desc) {
        set_error("null argument");
        return FM_E_INVALID;
    }
    fm_problem p;
    p.desc = *desc;
    std::string e = setup_problem(&p);
    if (!e.empty()) {
        set_error(e);
        return FM_E_INVALID;
    }
    HostFactors hf;
    e = build_factors(&p, hf);
    if (!e.empty()) {
        set_error(e);
        return FM_E_PENCIL;
    }
    int pairs = 0;
    for (int a = 0; a < 3; ++a) {
        for (auto t : hf.comp[a].tx) pairs += (t == 1);
        for (auto t : hf.comp[a].ty) pairs += (t == 1);
    }
    if (max_err) *max_err = hf.max_err;
    if (complex_pairs) *complex_pairs = pairs;
    if (n_unknowns) *n_unknowns = size_t(p.N);
    return FM_OK;
}

fm_status fm_host_coupling(const fm_problem_desc *desc, const double *x, double *y, long long *npairs, int *ntasks) {
    if (!desc) {
        set_error("null argument");
        return FM_E_INVALID;
    }
    fm_problem p;
    p.desc = *desc;
    std::string e = setup_problem(&p);
    if (!e.empty()) {
        set_error(e);
        return FM_E_INVALID;
    }
    HostFactors hf;
    e = build_factors(&p, hf);
    if (!e.empty()) {
        set_error(e);
        return FM_E_PENCIL;
    }
    CouplingHost ch;
    e = build_coupling(&p, hf, ch);
    if (!e.empty()) {
        set_error(e);
        return FM_E_INVALID;
    }
    if (npairs) *npairs = ch.npairs;
    if (ntasks) *ntasks = ch.ntasks;
    if (!x || !y) return FM_OK;
    const int nM = p.nM;
    const long long N = p.N, np = ch.npairs;
    std::vector<double> c0(N, 0.0), c1(N, 0.0);
    auto shapes = [](int q, double s, double r, double *v) {
        const double s2 = s * s, s3 = s2 * s;
        if (q == 2) {
            v[0] = 1.0 - 3.0 * s2 + 2.0 * s3;
            v[1] = r * (s - 2.0 * s2 + s3);
            v[2] = 3.0 * s2 - 2.0 * s3;
            v[3] = r * (s3 - s2);
        } else {
            const double s4 = s3 * s, s5 = s4 * s, r2 = r * r;
            v[0] = 1.0 - 10.0 * s3 + 15.0 * s4 - 6.0 * s5;
            v[1] = r * (s - 6.0 * s3 + 8.0 * s4 - 3.0 * s5);
            v[2] = r2 * 0.5 * (s2 - 3.0 * s3 + 3.0 * s4 - s5);
            v[3] = 10.0 * s3 - 15.0 * s4 + 6.0 * s5;
            v[4] = r * (-4.0 * s3 + 7.0 * s4 - 3.0 * s5);
            v[5] = r2 * 0.5 * (s3 - 2.0 * s4 + s5);
        }
    };
    // one pair as a coupling kernel lane evaluates it, from the task record the
    // lane reads (function indices, beta's sizes and offset, the task index for
    // the cell widths)
    std::vector<unsigned char> seen(size_t(np), 0);
    auto eval_pair = [&](const int *tk, long long pr) {
        const int b = tk[CT_BETA], task = tk[CT_TASK];
        const int bnx = tk[CT_NX], bny = tk[CT_NY], bnpts = tk[CT_NPTS];
        const long long boff = (long long)(((unsigned long long)(unsigned)tk[CT_OFF_HI] << 32) | (unsigned)tk[CT_OFF_LO]);
        const int qz = p.bz[b].q, qx = p.bx[b].q, qy = p.by[b].q;
        const int *gz = tk + CT_FIDX, *gx = gz + 2 * qz, *gy = gx + 2 * qx;
        double vz[MAXR], vx[MAXR], vy[MAXR];
        shapes(qz, ch.s[pr], ch.r[3 * size_t(task)], vz);
        shapes(qx, ch.s[np + pr], ch.r[3 * size_t(task) + 1], vx);
        shapes(qy, ch.s[2 * np + pr], ch.r[3 * size_t(task) + 2], vy);
        double val[MAXM];
        for (int jM = 0; jM < nM; ++jM) {
            const double *cb = x + boff + (long long)jM * bnpts;
            double acc = 0;
            for (int cz = 0; cz < 2 * qz; ++cz) {
                if (gz[cz] < 0) continue;
                double accx = 0;
                for (int ax = 0; ax < 2 * qx; ++ax) {
                    if (gx[ax] < 0) continue;
                    double accy = 0;
                    for (int ay = 0; ay < 2 * qy; ++ay)
                        if (gy[ay] >= 0) accy += vy[ay] * cb[((long long)gz[cz] * bnx + gx[ax]) * bny + gy[ay]];
                    accx += vx[ax] * accy;
                }
                acc += vz[cz] * accx;
            }
            val[jM] = acc;
        }
        const int o = ch.out[pr], outp = o >> 1, slot = o & 1;
        const int a = outp >= p.off[2] ? 2 : (outp >= p.off[1] ? 1 : 0);
        std::vector<double> &dst = slot == 0 ? c0 : c1;
        for (int iM = 0; iM < nM; ++iM) {
            double v = 0;
            for (int jM = 0; jM < nM; ++jM) v += ch.F[size_t(iM * nM + jM) * np + pr] * val[jM];
            dst[outp + (long long)iM * p.npts[a]] = v;
        }
        ++seen[pr];
    };
    // the pairs in the kernels' order: per wave job and lane, the record the
    // lane reads and the pair(s) it takes
    if (nM == 1) {
        const int P = ch.pairs_per_lane;
        for (int j = 0; j < ch.njobs; ++j) {
            const bool split = P == 2 || ch.jrec[size_t(2 * j) * CPL_TASK + CT_SPLIT] != 0;
            for (int lane = 0; lane < 64; ++lane) {
                const int *tk = &ch.jrec[size_t(2 * j + (lane >> 5)) * CPL_TASK];
                const int W = split ? 32 : 64, li = split ? lane & 31 : lane;
                for (int q = 0; q < P; ++q)
                    if (li + W * q < tk[CT_COUNT]) eval_pair(tk, tk[CT_FIRST] + li + W * q);
            }
        }
    } else {
        for (int j = 0; j < ch.njobs; ++j) {
            const int *tk = &ch.task[size_t(j) * CPL_TASK];
            for (int lane = 0; lane < 64; ++lane)
                if (lane < tk[CT_COUNT]) eval_pair(tk, tk[CT_FIRST] + lane);
        }
    }
    for (long long pr = 0; pr < np; ++pr)
        if (seen[pr] != 1) {
            set_error("coupling jobs do not take every pair exactly once");
            return FM_E_INVALID;
        }
    for (long long i = 0; i < N; ++i) y[i] = c0[i] + c1[i];
    return FM_OK;
}

fm_status fm_host_precond(const fm_problem_desc *desc, double E, const double *r, double *z) {
    if (!desc || !r || !z) {
        set_error("null argument");
        return FM_E_INVALID;
    }
    fm_problem p;
    p.desc = *desc;
    std::string e = setup_problem(&p);
    if (!e.empty()) {
        set_error(e);
        return FM_E_INVALID;
    }
    HostFactors hf;
    e = build_factors(&p, hf);
    if (!e.empty()) {
        set_error(e);
        return FM_E_PENCIL;
    }
    const int nM = p.nM;
    for (int a = 0; a < 3; ++a) {
        if (p.absent(a)) continue;
        const HostComp &h = hf.comp[a];
        for (auto t : h.tx)
            if (t) {
                set_error("complex pencil pairs are not handled by the host apply");
                return FM_E_PENCIL;
            }
        for (auto t : h.ty)
            if (t) {
                set_error("complex pencil pairs are not handled by the host apply");
                return FM_E_PENCIL;
            }
        const int nx = p.bx[a].n, ny = p.by[a].n, nz = p.bz[a].n, nxy = nx * ny, n = nM * nz;
        const double *ra = r + p.off[a];
        double *za = z + p.off[a];
        // z transform: rows (iM, k) -> slots
        std::vector<double> t(size_t(n) * nxy, 0.0);
        for (int s = 0; s < n; ++s)
            for (int q = 0; q < n; ++q) {
                double w;
                if (p.variant == 2) {
                    w = h.Zj[size_t(s) * n + q];
                } else {
                    const int iM = s / nz, k = s % nz;
                    if (q / nz != iM) continue;
                    w = h.Wz[size_t(iM) * 2 * nz * nz + size_t(k) * nz + q % nz];
                }
                if (w == 0.0) continue;
                for (int c = 0; c < nxy; ++c) t[size_t(s) * nxy + c] += w * ra[size_t(q) * nxy + c];
            }
        // per slot: X = Wbar_x T Wbar_y^T, divide, T = W_x X W_y^T
        std::vector<double> X(static_cast<size_t>(nxy));
        for (int s = 0; s < n; ++s) {
            double *T = t.data() + size_t(s) * nxy;
            const double *Wbx = h.Wx.data() + size_t(s) * 2 * nx * nx, *Wx = Wbx + size_t(nx) * nx;
            const double *Wby = h.Wy.data() + size_t(s) * 2 * ny * ny, *Wy = Wby + size_t(ny) * ny;
            const double *lx = h.lx.data() + size_t(s) * nx, *ly = h.ly.data() + size_t(s) * ny;
            auto prod = [&](const double *L, const double *R, const double *in, double *out) {
                for (int i = 0; i < nx; ++i)
                    for (int j = 0; j < ny; ++j) {
                        double v = 0;
                        for (int i2 = 0; i2 < nx; ++i2) {
                            double u = 0;
                            for (int j2 = 0; j2 < ny; ++j2) u += in[size_t(i2) * ny + j2] * R[size_t(j) * ny + j2];
                            v += L[size_t(i) * nx + i2] * u;
                        }
                        out[size_t(i) * ny + j] = v;
                    }
            };
            prod(Wbx, Wby, T, X.data());
            for (int i = 0; i < nx; ++i)
                for (int j = 0; j < ny; ++j) X[size_t(i) * ny + j] /= lx[i] + ly[j] - E;
            prod(Wx, Wy, X.data(), T);
        }
        // back: slots -> rows (iM, k)
        for (size_t i = 0; i < size_t(n) * nxy; ++i) za[i] = 0.0;
        for (int q = 0; q < n; ++q)
            for (int s = 0; s < n; ++s) {
                double w;
                if (p.variant == 2) {
                    w = h.Zj[size_t(n) * n + size_t(q) * n + s];
                } else {
                    const int iM = q / nz, k = q % nz;
                    if (s / nz != iM) continue;
                    w = h.Wz[size_t(iM) * 2 * nz * nz + size_t(nz) * nz + size_t(k) * nz + s % nz];
                }
                if (w == 0.0) continue;
                for (int c = 0; c < nxy; ++c) za[size_t(q) * nxy + c] += w * t[size_t(s) * nxy + c];
            }
    }
    return FM_OK;
}

}  // extern "C"

fm_status fm_host_slice_eigenvalues(const fm_problem_desc *desc, int alpha, int slot, double *lx_re, double *lx_im,
                                    double *ly_re, double *ly_im) {
    if (!desc) {
        set_error("null argument");
        return FM_E_INVALID;
    }
    fm_problem p;
    p.desc = *desc;
    std::string e = setup_problem(&p);
    if (!e.empty()) {
        set_error(e);
        return FM_E_INVALID;
    }
    if (alpha < 0 || alpha > 2 || p.absent(alpha) || slot < 0 || slot >= p.nM * p.bz[alpha].n) {
        set_error("alpha or slot out of range");
        return FM_E_INVALID;
    }
    HostFactors hf;
    e = build_factors(&p, hf);
    if (!e.empty()) {
        set_error(e);
        return FM_E_PENCIL;
    }
    const HostComp &h = hf.comp[alpha];
    const int nx = p.bx[alpha].n, ny = p.by[alpha].n;
    for (int i = 0; i < nx; ++i) {
        if (lx_re) lx_re[i] = h.lx[size_t(slot) * nx + i];
        if (lx_im) lx_im[i] = h.lxi[size_t(slot) * nx + i];
    }
    for (int i = 0; i < ny; ++i) {
        if (ly_re) ly_re[i] = h.ly[size_t(slot) * ny + i];
        if (ly_im) ly_im[i] = h.lyi[size_t(slot) * ny + i];
    }
    return FM_OK;
}

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

}  // extern "C"

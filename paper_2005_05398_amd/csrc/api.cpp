// C ABI of the FM solver (include/fm.h): problem creation and upload,
// operator and preconditioner application, batched flexible GMRES.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "batch.h"
#include "fm_problem.h"

namespace fm {

namespace {
thread_local std::string g_err;

fm_status fail(fm_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(FM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
const T *put(fm_problem *p, const std::vector<T> &h, std::string &err) {
    if (h.empty()) return nullptr;
    void *d = nullptr;
    size_t bytes = h.size() * sizeof(T);
    if (hipMalloc(&d, bytes) != hipSuccess) {
        err = "device allocation failed";
        return nullptr;
    }
    p->buffers.push_back({d, bytes});
    p->bytes_resident += bytes;
    if (hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        err = "device copy failed";
        return nullptr;
    }
    return static_cast<const T *>(d);
}

DimDev dim_dev(fm_problem *p, const Basis1D &b, std::string &err) {
    DimDev d;
    d.n = b.n;
    d.K = b.K;
    d.q = b.q;
    d.drop0 = b.dirichlet ? 1 : 0;
    d.R = b.nodes.back();
    d.lo = b.lo;
    d.hbar = b.hbar;
    d.nodes = put(p, b.nodes, err);
    d.pts = put(p, b.points, err);
    d.idx = put(p, b.idx, err);
    d.S = put(p, b.val[0], err);
    d.D1 = put(p, b.val[1], err);
    d.D2 = put(p, b.val[2], err);
    std::vector<int> lo(b.n), hi(b.n);
    for (int i = 0; i < b.n; ++i) {
        lo[i] = 1 << 30;
        hi[i] = -1;
        for (int s = 0; s < MAXR; ++s) {
            int g = b.idx[size_t(i) * MAXR + s];
            if (g >= 0) {
                lo[i] = std::min(lo[i], g);
                hi[i] = std::max(hi[i], g);
            }
        }
    }
    d.first = put(p, lo, err);
    d.last = put(p, hi, err);
    return d;
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// bfloat16 round to nearest even, and back
unsigned short bf16_rne(float f) {
    unsigned u;
    std::memcpy(&u, &f, 4);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
float bf16_value(unsigned short h) {
    unsigned u = unsigned(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Small per-call device arrays: energies, flags, minimum denominators.
struct Small {
    double *E, *min_den;
    int *running, *mask;
};

fm_status ensure_small(fm_problem *p, int nb, Small &s) {
    size_t need = round256(sizeof(double) * nb) * 2 + round256(sizeof(int) * nb) * 2;
    if (p->ws_small_bytes < need) {
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        if (p->ws_small) (void)hipFree(p->ws_small);
        p->ws_small = nullptr;
        p->ws_small_bytes = 0;
        HIP_TRY(hipMalloc(&p->ws_small, need));
        p->ws_small_bytes = need;
    }
    char *c = static_cast<char *>(p->ws_small);
    s.E = reinterpret_cast<double *>(c);
    c += round256(sizeof(double) * nb);
    s.min_den = reinterpret_cast<double *>(c);
    c += round256(sizeof(double) * nb);
    s.running = reinterpret_cast<int *>(c);
    c += round256(sizeof(int) * nb);
    s.mask = reinterpret_cast<int *>(c);
    return FM_OK;
}

fm_status ensure_pinned(fm_problem *p, size_t bytes) {
    if (p->host_pinned_bytes >= bytes) return FM_OK;
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    if (p->host_pinned) (void)hipHostFree(p->host_pinned);
    p->host_pinned = nullptr;
    p->host_pinned_bytes = 0;
    void *h = nullptr;
    HIP_TRY(hipHostMalloc(&h, bytes, hipHostMallocDefault));
    p->host_pinned = static_cast<double *>(h);
    p->host_pinned_bytes = bytes;
    return FM_OK;
}

size_t krylov_bytes(long long N, int nb, int m) {
    size_t b = 0;
    b += round256(sizeof(double) * size_t(m + 1) * nb * N);   // V
    b += round256(sizeof(double) * size_t(m) * nb * N);       // Z
    b += round256(sizeof(double) * size_t(nb) * (m + 1) * m); // H
    b += 4 * round256(sizeof(double) * size_t(nb) * (m + 1)); // g, hcol, hproj, y
    b += 2 * round256(sizeof(double) * size_t(nb) * m);       // cs, sn
    b += round256(sizeof(double) * size_t(nb) * (2 * m + 3) * NBLK);
    b += 6 * round256(sizeof(double) * nb);                   // bnorm rnorm scal rho E tol
    b += 5 * round256(sizeof(int) * nb);                      // ticket active jcount flags closed
    return b;
}

// Lays the Krylov arrays out in one allocation starting at c.
char *carve_krylov(char *c, long long N, int nb, int m, KrylovDev &K) {
    auto take = [&](size_t bytes) {
        char *r = c;
        c += round256(bytes);
        return r;
    };
    K.nb = nb;
    K.m = m;
    K.N = N;
    K.V = (double *)take(sizeof(double) * size_t(m + 1) * nb * N);
    K.Z = (double *)take(sizeof(double) * size_t(m) * nb * N);
    K.H = (double *)take(sizeof(double) * size_t(nb) * (m + 1) * m);
    K.g = (double *)take(sizeof(double) * size_t(nb) * (m + 1));
    K.hcol = (double *)take(sizeof(double) * size_t(nb) * (m + 1));
    K.hproj = (double *)take(sizeof(double) * size_t(nb) * (m + 1));
    K.y = (double *)take(sizeof(double) * size_t(nb) * (m + 1));
    K.cs = (double *)take(sizeof(double) * size_t(nb) * m);
    K.sn = (double *)take(sizeof(double) * size_t(nb) * m);
    K.part = (double *)take(sizeof(double) * size_t(nb) * (2 * m + 3) * NBLK);
    K.bnorm = (double *)take(sizeof(double) * nb);
    K.rnorm = (double *)take(sizeof(double) * nb);
    K.scal = (double *)take(sizeof(double) * nb);
    K.rho = (double *)take(sizeof(double) * nb);
    K.E = (double *)take(sizeof(double) * nb);
    K.tol = (double *)take(sizeof(double) * nb);
    K.ticket = (unsigned *)take(sizeof(int) * nb);
    K.active = (int *)take(sizeof(int) * nb);
    K.jcount = (int *)take(sizeof(int) * nb);
    K.flags = (int *)take(sizeof(int) * nb);
    K.closed = (int *)take(sizeof(int) * nb);
    return c;
}

// -- per-kernel-class timing ---------------------------------------------
// Set while this thread enqueues work under stream capture: no events then.
thread_local bool t_capturing = false;

size_t prof_mark(fm_problem *p, hipStream_t st) {
    Profile &pf = p->prof;
    if (!pf.on || t_capturing) return SIZE_MAX;
    if (pf.next == pf.ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return SIZE_MAX;
        pf.ev.push_back(e);
    }
    if (hipEventRecord(pf.ev[pf.next], st) != hipSuccess) return SIZE_MAX;
    return pf.next++;
}

template <class F>
void timed(fm_problem *p, hipStream_t st, int cls, F &&f) {
    size_t a = prof_mark(p, st);
    f();
    size_t b = prof_mark(p, st);
    if (a != SIZE_MAX && b != SIZE_MAX) p->prof.recs.push_back({cls, a, b});
}

void prof_work(fm_problem *p, int cls, double bytes, double flops) {
    if (!p->prof.on) return;
    p->prof.bytes[cls] += bytes;
    p->prof.flops[cls] += flops;
}

// Reads the elapsed times of the recorded launches; the stream must be idle.
void prof_collect(fm_problem *p) {
    Profile &pf = p->prof;
    for (auto &r : pf.recs) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, pf.ev[r.e0], pf.ev[r.e1]) == hipSuccess) pf.ms[r.cls] += ms;
        pf.launches[r.cls] += 1;
    }
    pf.recs.clear();
    pf.next = 0;
}

// Algorithmic work of one request (unique FP64 words of each operation's definition).
struct Work {
    double N, pts, xyflops, localflops, coupflops, zflops;
    explicit Work(const fm_problem *p) {
        N = double(p->N);
        pts = double(p->npts[0] + p->npts[1] + p->npts[2]);
        xyflops = 0;
        zflops = 0;
        localflops = 0;
        coupflops = 0;
        const int nM = p->nM;
        for (int a = 0; a < 3; ++a) {
            const double np = double(p->npts[a]);
            xyflops += 4.0 * nM * p->bz[a].n * double(p->bx[a].n) * p->by[a].n * (p->bx[a].n + p->by[a].n);
            // one z product per direction: n_z (block-Jacobi) or n_M n_z (joint) terms per unknown
            zflops += 2.0 * 2.0 * (p->variant == 2 ? nM * p->bz[a].n : p->bz[a].n) * nM * np;
            // local stencil as separable banded passes: 9 passes of 2q terms (2 flops each) per
            // unknown, plus the pointwise combination (about 20 flops) and the M'+-1 terms
            const double r = 2.0 * std::max(p->bx[a].q, std::max(p->by[a].q, p->bz[a].q));
            localflops += np * nM * (9 * 2 * r + 20 + (nM > 1 ? 12 : 0));
            // coupling: per beta the r_z r_x r_y contraction (2 flops each) for each M'', plus
            // the M'' -> M' weights
            for (int b = 0; b < 3; ++b)
                if (b != a)
                    coupflops += np * (nM * 2.0 * (2 * p->bz[b].q) * (2 * p->bx[b].q) * (2 * p->by[b].q) +
                                       2.0 * nM * nM);
        }
    }
    // a complex request: two real rows (both parts), every operation's work twice
    // (the E_i S term of its operator is not counted)
    Work &rows(int r) {
        N *= r;
        pts *= r;
        xyflops *= r;
        zflops *= r;
        localflops *= r;
        coupflops *= r;
        return *this;
    }
    double matvec() const { return 8 * (2 * N + pts); }
    double coupling() const { return 8 * 3 * N; }
    double modez() const { return 8 * 2 * N; }
    double xy() const { return 8 * 2 * N; }
    // Arnoldi step j: the dot pass reads Q (j vectors), U and W; the update pass
    // reads them too and writes U and W
    double dots(int j) const { return 8 * (j + 2) * N; }
    double update(int j) const { return 8 * (j + 4) * N; }
};

void add_precond_work(fm_problem *p, const Work &w, double nreq) {
    prof_work(p, FM_K_MODEZ, 2 * w.modez() * nreq, w.zflops * nreq);
    prof_work(p, FM_K_XY, w.xy() * nreq, w.xyflops * nreq);
}

void add_matvec_work(fm_problem *p, const Work &w, double nreq) {
    prof_work(p, FM_K_MATVEC, w.matvec() * nreq, w.localflops * nreq);
    prof_work(p, FM_K_COUPLING, w.coupling() * nreq, w.coupflops * nreq);
}

void apply_operator(fm_problem *p, int nb, const double *E_dev, const int *mask, const double *x, double *y,
                    double *cbuf, hipStream_t st) {
    timed(p, st, FM_K_COUPLING, [&] { launch_matvec(p->pd, nb, E_dev, mask, x, y, cbuf, st, 2); });
    timed(p, st, FM_K_MATVEC, [&] { launch_matvec(p->pd, nb, E_dev, mask, x, y, cbuf, st, 1); });
}

// Work of Arnoldi step j for one request: update = false for the step on which
// the request met its tolerance (no update pass follows).
void add_step_work(fm_problem *p, const Work &w, int j, bool update) {
    add_precond_work(p, w, 1);
    add_matvec_work(p, w, 1);
    prof_work(p, FM_K_MDOT, w.dots(j), 2.0 * (2 * j + 2) * w.N);
    prof_work(p, FM_K_FINISH, 0, 6.0 * j + 4.0 * j);
    if (update) prof_work(p, FM_K_MUPDATE, w.update(j), (4.0 * j + 4) * w.N);
}

// Closing pass after `steps` steps: dots over Q and U only, then the finish.
void add_closing_work(fm_problem *p, const Work &w, int steps) {
    prof_work(p, FM_K_MDOT, 8.0 * (steps + 1) * w.N, 2.0 * (steps + 1) * w.N);
    prof_work(p, FM_K_FINISH, 0, 10.0 * steps);
}

// tmp: [nb][N] scratch for the staged x-y products (may be null).
void apply_precond(fm_problem *p, int nb, const double *E_dev, const int *mask, const double *in, double *out,
                   int prec, double *min_den, double *tmp, hipStream_t st) {
    if (prec != FM_FP64 && precond_f32_ok(p->pd, p->pr, nb, prec)) {
        // FP32 storage between the reduced-precision products
        timed(p, st, FM_K_MODEZ, [&] { launch_z_f32(p->pd, p->pr, nb, mask, 0, in, out, tmp, st); });
        timed(p, st, FM_K_XY, [&] { launch_xy_f32(p->pd, p->pr, nb, E_dev, mask, prec, out, tmp, st); });
        timed(p, st, FM_K_MODEZ, [&] { launch_z_f32(p->pd, p->pr, nb, mask, 1, in, out, tmp, st); });
        return;
    }
    if (p->pr.coupled) {
        // joint z transform into tmp, the x-y slots in place there (out as their
        // scratch: in is no longer needed), joint z transform back into out
        timed(p, st, FM_K_MODEZ, [&] { launch_zjoint(p->pd, p->pr, nb, mask, 0, in, tmp, st); });
        bool ok = false;
        if (prec != FM_FP64)
            timed(p, st, FM_K_XY, [&] { ok = launch_xy_lp(p->pd, p->pr, nb, E_dev, mask, tmp, prec, out, st); });
        if (!ok) timed(p, st, FM_K_XY, [&] { launch_xy(p->pd, p->pr, nb, E_dev, mask, tmp, min_den, out, st); });
        timed(p, st, FM_K_MODEZ, [&] { launch_zjoint(p->pd, p->pr, nb, mask, 1, tmp, out, st); });
        return;
    }
    if (prec != FM_FP64) {
        bool ok = true;
        timed(p, st, FM_K_MODEZ, [&] { launch_modez_lp(p->pd, p->pr, nb, mask, 0, in, out, st); });
        timed(p, st, FM_K_XY, [&] { ok = launch_xy_lp(p->pd, p->pr, nb, E_dev, mask, out, prec, tmp, st); });
        if (!ok) timed(p, st, FM_K_XY, [&] { launch_xy(p->pd, p->pr, nb, E_dev, mask, out, min_den, tmp, st); });
        timed(p, st, FM_K_MODEZ, [&] { launch_modez_lp(p->pd, p->pr, nb, mask, 1, out, out, st); });
        return;
    }
    timed(p, st, FM_K_MODEZ, [&] { launch_modez(p->pd, p->pr, nb, mask, 0, in, out, st); });
    timed(p, st, FM_K_XY, [&] { launch_xy(p->pd, p->pr, nb, E_dev, mask, out, min_den, tmp, st); });
    timed(p, st, FM_K_MODEZ, [&] { launch_modez(p->pd, p->pr, nb, mask, 1, out, out, st); });
}

// Complex energies (rows 2c, 2c + 1 = real and imaginary part of complex
// request c): (H - E S) x = A(Re E) x + i Im E ... applied as A(Re E) on both
// rows, then y_re += Im E (S x)_im, y_im -= Im E (S x)_re.  E2: Re E per row;
// active: per complex request, mask2 the same per row (both may be null);
// tmp: [2 nbc][N] scratch for S x.
void apply_operator_complex(fm_problem *p, int nbc, const double *E2, const double *Eim, const int *active,
                            const int *mask2, const double *x, double *y, double *cbuf, double *tmp,
                            hipStream_t st) {
    apply_operator(p, 2 * nbc, E2, mask2, x, y, cbuf, st);
    timed(p, st, FM_K_MATVEC, [&] {
        launch_mass(p->pd, 2 * nbc, x, tmp, st, mask2);
        launch_cplx_energy(y, tmp, Eim, active, nbc, p->N, st);
    });
}

// z = L(E)^-1 r with E complex: the real z and x-y transforms on both rows,
// the complex divide between the forward and backward x-y products (FP64).
// tmp: [2 nbc][N] scratch.
void apply_precond_complex(fm_problem *p, int nbc, const double *Ere, const double *Eim, const int *active,
                           const int *mask2, const double *in, double *out, double *min_den, double *tmp,
                           hipStream_t st) {
    const int nr = 2 * nbc;
    if (p->pr.coupled) {
        timed(p, st, FM_K_MODEZ, [&] { launch_zjoint(p->pd, p->pr, nr, mask2, 0, in, tmp, st); });
        timed(p, st, FM_K_XY, [&] {
            launch_xy_half(p->pd, p->pr, nr, mask2, 0, tmp, out, st);
            launch_cdivide(p->pd, p->pr, nbc, Ere, Eim, active, tmp, min_den, st);
            launch_xy_half(p->pd, p->pr, nr, mask2, 1, tmp, out, st);
        });
        timed(p, st, FM_K_MODEZ, [&] { launch_zjoint(p->pd, p->pr, nr, mask2, 1, tmp, out, st); });
        return;
    }
    timed(p, st, FM_K_MODEZ, [&] { launch_modez(p->pd, p->pr, nr, mask2, 0, in, out, st); });
    timed(p, st, FM_K_XY, [&] {
        launch_xy_half(p->pd, p->pr, nr, mask2, 0, out, tmp, st);
        launch_cdivide(p->pd, p->pr, nbc, Ere, Eim, active, out, min_den, st);
        launch_xy_half(p->pd, p->pr, nr, mask2, 1, out, tmp, st);
    });
    timed(p, st, FM_K_MODEZ, [&] { launch_modez(p->pd, p->pr, nr, mask2, 1, out, out, st); });
}

}  // namespace

// -- Batch -----------------------------------------------------------------

size_t Batch::footprint(const fm_problem *p, int cap, int m, int cplx) {
    const long long Nv = cplx ? 2 * p->N : p->N;
    return krylov_bytes(Nv, cap, m) + 3 * round256(sizeof(int) * cap) + round256(sizeof(double) * cap) +
           round256(sizeof(double) * 2 * size_t(cap) * size_t(Nv)) + round256(sizeof(double) * size_t(cap) * size_t(Nv)) +
           (cplx ? round256(sizeof(double) * 2 * cap) + round256(sizeof(double) * cap) + round256(sizeof(int) * 2 * cap)
                 : 0);
}

fm_status Batch::create(fm_problem *pp, int c, int mm, hipStream_t s, int cx) {
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    p = pp;
    cap = c;
    m = mm;
    st = s;
    cplx = cx;
    const long long Nv = cplx ? 2 * p->N : p->N;
    bytes = footprint(p, cap, m, cplx);
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        mem = nullptr;
        return fail(FM_E_NOMEM, "Krylov workspace allocation failed");
    }
    char *q = carve_krylov(static_cast<char *>(mem), Nv, cap, m, K);
    running = reinterpret_cast<int *>(q);
    q += round256(sizeof(int) * cap);
    cont = reinterpret_cast<int *>(q);
    q += round256(sizeof(int) * cap);
    fresh = reinterpret_cast<int *>(q);
    q += round256(sizeof(int) * cap);
    min_den = reinterpret_cast<double *>(q);
    q += round256(sizeof(double) * cap);
    cbuf = reinterpret_cast<double *>(q);
    q += round256(sizeof(double) * 2 * size_t(cap) * size_t(Nv));
    ptmp = reinterpret_cast<double *>(q);
    if (cplx) {
        q += round256(sizeof(double) * size_t(cap) * size_t(Nv));
        E2 = reinterpret_cast<double *>(q);
        q += round256(sizeof(double) * 2 * cap);
        Eim = reinterpret_cast<double *>(q);
        q += round256(sizeof(double) * cap);
        mask2 = reinterpret_cast<int *>(q);
    }
    void *h = nullptr;
    HIP_TRY(hipHostMalloc(&h, sizeof(int) * cap, hipHostMallocDefault));
    hbuf = static_cast<int *>(h);
    // zero everything but the Krylov bases and the preconditioner scratch, which
    // are written before they are read (the coupling buffer must start at zero)
    {
        char *z0 = reinterpret_cast<char *>(K.H);
        char *z1 = reinterpret_cast<char *>(ptmp);
        HIP_TRY(hipMemsetAsync(z0, 0, size_t(z1 - z0), st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    run.assign(cap, 0);
    iters.assign(cap, 0);
    restarts.assign(cap, 0);
    limit.assign(cap, 1 << 30);
    last_steps.assign(cap, 0);
    E.assign(cap, 0.0);
    Ei.assign(cap, 0.0);
    return FM_OK;
}

void Batch::release() {
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    for (hipGraphExec_t g : gexec)
        if (g) (void)hipGraphExecDestroy(g);
    gexec.clear();
    if (cap_st) (void)hipStreamDestroy(cap_st);
    cap_st = nullptr;
    if (mem) (void)hipFree(mem);
    if (hbuf) (void)hipHostFree(hbuf);
    mem = nullptr;
    hbuf = nullptr;
}

void Batch::enqueue_step(int j, hipStream_t s, bool profile) {
    const int nb = cap;
    const long long N = K.N;
    double *Vj = K.V + (long long)j * nb * N;
    double *Zj = K.Z + (long long)j * nb * N;
    double *Vn = K.V + (long long)(j + 1) * nb * N;
    if (cplx) {
        t_capturing = !profile;
        launch_expand_mask(K.active, mask2, nb, s);
        apply_precond_complex(p, nb, K.E, Eim, K.active, mask2, Vj, Zj, min_den, ptmp, s);
        apply_operator_complex(p, nb, E2, Eim, K.active, mask2, Zj, Vn, cbuf, ptmp, s);
        t_capturing = false;
        if (profile) {
            timed(p, s, FM_K_MDOT, [&] { launch_arnoldi_dots(K, j, 0, s); });
            timed(p, s, FM_K_FINISH, [&] { launch_arnoldi_finish(K, j, 0, s); });
            timed(p, s, FM_K_MUPDATE, [&] { launch_arnoldi_update(K, j, s); });
        } else {
            launch_arnoldi_dots(K, j, 0, s);
            launch_arnoldi_finish(K, j, 0, s);
            launch_arnoldi_update(K, j, s);
        }
        return;
    }
    if (profile) {
        apply_precond(p, nb, K.E, K.active, Vj, Zj, prec, min_den, ptmp, s);
        apply_operator(p, nb, K.E, K.active, Zj, Vn, cbuf, s);
        timed(p, s, FM_K_MDOT, [&] { launch_arnoldi_dots(K, j, 0, s); });
        timed(p, s, FM_K_FINISH, [&] { launch_arnoldi_finish(K, j, 0, s); });
        timed(p, s, FM_K_MUPDATE, [&] { launch_arnoldi_update(K, j, s); });
        return;
    }
    // the same launches without the profiling events (used under capture)
    t_capturing = true;
    apply_precond(p, nb, K.E, K.active, Vj, Zj, prec, min_den, ptmp, s);
    apply_operator(p, nb, K.E, K.active, Zj, Vn, cbuf, s);
    t_capturing = false;
    launch_arnoldi_dots(K, j, 0, s);
    launch_arnoldi_finish(K, j, 0, s);
    launch_arnoldi_update(K, j, s);
}

hipGraphExec_t Batch::step_graph(int j0, int n) {
    const int groups = (m + GRAPH_STEPS - 1) / GRAPH_STEPS;
    if (gexec.empty()) gexec.assign(size_t(3) * groups, nullptr);
    const size_t idx = size_t(prec) * groups + j0 / GRAPH_STEPS;
    if (gexec[idx]) return gexec[idx];
    if (graphs_failed) return nullptr;
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    if (!cap_st && hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking) != hipSuccess) {
        cap_st = nullptr;
        graphs_failed = true;
        return nullptr;
    }
    (void)hipGetLastError();
    if (hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed) != hipSuccess) {
        graphs_failed = true;
        return nullptr;
    }
    for (int j = j0; j < j0 + n; ++j) enqueue_step(j, cap_st, false);
    hipGraph_t g = nullptr;
    const hipError_t e_end = hipStreamEndCapture(cap_st, &g);
    hipGraphExec_t ex = nullptr;
    if (e_end != hipSuccess || !g || hipGetLastError() != hipSuccess ||
        hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        ex = nullptr;
        graphs_failed = true;        // this batch launches eagerly from now on
        (void)hipGetLastError();     // a failed capture must not fail the next checked call
    }
    if (g) (void)hipGraphDestroy(g);
    gexec[idx] = ex;
    return ex;
}

bool Batch::any_running() const {
    for (int v : run)
        if (v) return true;
    return false;
}

fm_status Batch::boundary(const std::vector<int> &joining, int x0_is_guess) {
    std::vector<int> hcont(run), hfresh(cap, 0);
    bool any_cont = false, any_fresh = !joining.empty();
    for (int v : hcont) any_cont |= v != 0;
    std::vector<double> big(cap, 1e300);
    for (int s : joining) {
        hfresh[s] = 1;
        run[s] = 1;
        iters[s] = 0;
        restarts[s] = 0;
    }
    HIP_TRY(hipMemcpyAsync(K.E, E.data(), sizeof(double) * cap, hipMemcpyHostToDevice, st));
    std::vector<double> e2;
    if (cplx) {
        e2.resize(2 * size_t(cap));
        for (int s = 0; s < cap; ++s) e2[2 * s] = e2[2 * s + 1] = E[s];
        HIP_TRY(hipMemcpyAsync(E2, e2.data(), sizeof(double) * 2 * cap, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(Eim, Ei.data(), sizeof(double) * cap, hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipMemcpyAsync(cont, hcont.data(), sizeof(int) * cap, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(fresh, hfresh.data(), sizeof(int) * cap, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(running, run.data(), sizeof(int) * cap, hipMemcpyHostToDevice, st));
    if (any_fresh) {
        // per-slot reset of flags and minimum denominators
        std::vector<int> zero_flags(cap, 0);
        HIP_TRY(hipMemcpyAsync(hbuf, K.flags, sizeof(int) * cap, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::vector<double> md(cap);
        HIP_TRY(hipMemcpyAsync(md.data(), min_den, sizeof(double) * cap, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int s : joining) {
            hbuf[s] = 0;
            md[s] = 1e300;
        }
        HIP_TRY(hipMemcpyAsync(K.flags, hbuf, sizeof(int) * cap, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(min_den, md.data(), sizeof(double) * cap, hipMemcpyHostToDevice, st));
    }
    timed(p, st, FM_K_RESTART, [&] {
        if (any_cont) {
            launch_cycle_solve(K, cont, st);
            launch_xupdate(K, cont, X, st);
        }
        if (any_fresh) {
            launch_zero_start(K, X, fresh, x0_is_guess ? 0 : 1, st);
            launch_bnorm(K, B, fresh, st);
        }
        if (cplx) {
            launch_expand_mask(running, mask2, cap, st);
            launch_matvec(p->pd, 2 * cap, E2, mask2, X, K.V, cbuf, st);
            launch_mass(p->pd, 2 * cap, X, ptmp, st, mask2);
            launch_cplx_energy(K.V, ptmp, Eim, running, cap, p->N, st);
        } else {
            launch_matvec(p->pd, cap, K.E, running, X, K.V, cbuf, st);
        }
        launch_residual(K, running, B, rtol, 0.5, st);
        launch_scale0(K, st);
    });
    HIP_TRY(hipGetLastError());
    if (any_cont) {
        Work w(p);
        w.rows(cplx ? 2 : 1);
        for (int s = 0; s < cap; ++s)
            if (hcont[s]) prof_work(p, FM_K_RESTART, 8.0 * (last_steps[s] + 2) * w.N + w.matvec() + 8 * 5 * w.N, 0);
    }
    HIP_TRY(hipMemcpyAsync(hbuf, running, sizeof(int) * cap, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    prof_collect(p);
    std::vector<int> over;
    for (int s = 0; s < cap; ++s) {
        run[s] = hbuf[s];
        if (run[s] && iters[s] >= limit[s]) over.push_back(s);
    }
    return stop(over);
}

fm_status Batch::stop(const std::vector<int> &slots) {
    if (slots.empty()) return FM_OK;
    for (int s : slots) run[s] = 0;
    HIP_TRY(hipMemcpyAsync(running, run.data(), sizeof(int) * cap, hipMemcpyHostToDevice, st));
    std::vector<int> act(cap);
    HIP_TRY(hipMemcpyAsync(act.data(), K.active, sizeof(int) * cap, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int s : slots) act[s] = 0;
    HIP_TRY(hipMemcpyAsync(K.active, act.data(), sizeof(int) * cap, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return FM_OK;
}

fm_status Batch::cycle(const std::function<bool()> &want_cut, int min_steps) {
    const int nb = cap;
    const int poll = GRAPH_STEPS;
    int steps = 0;
    for (int j = 0; j < m;) {
        const int n = std::min(poll, m - j);
        hipGraphExec_t g = (graphs && !p->prof.on) ? step_graph(j, n) : nullptr;
        if (g) {
            HIP_TRY(hipGraphLaunch(g, st));
        } else {
            for (int i = j; i < j + n; ++i) enqueue_step(i, st, p->prof.on);
        }
        j += n;
        steps = j;
        if (steps < m) {
            HIP_TRY(hipMemcpyAsync(hbuf, K.active, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            bool any = false;
            for (int i = 0; i < nb; ++i) any |= hbuf[i] != 0;
            if (!any) break;
            if (want_cut && steps >= min_steps && want_cut()) break;
        }
    }
    // the last column of the requests still iterating
    timed(p, st, FM_K_MDOT, [&] { launch_arnoldi_dots(K, steps, 1, st); });
    timed(p, st, FM_K_FINISH, [&] { launch_arnoldi_finish(K, steps, 1, st); });
    HIP_TRY(hipGetLastError());
    std::vector<int> closed(nb);
    HIP_TRY(hipMemcpyAsync(hbuf, K.jcount, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(closed.data(), K.closed, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    prof_collect(p);
    Work w(p);
    w.rows(cplx ? 2 : 1);
    for (int i = 0; i < nb; ++i)
        if (run[i]) {
            const int jc = hbuf[i];
            last_steps[i] = jc;
            if (p->prof.on) {
                for (int j = 0; j < jc; ++j) add_step_work(p, w, j, true);
                if (closed[i]) add_closing_work(p, w, jc);
                else add_step_work(p, w, jc, false);
            }
            iters[i] += std::max(1, jc);     // every cycle counts as progress
            restarts[i] += 1;
        }
    return FM_OK;
}

fm_status Batch::read_results(std::vector<double> &rel, std::vector<double> &mind, std::vector<int> &flags) {
    std::vector<double> rn(cap), bn(cap);
    mind.assign(cap, 0.0);
    flags.assign(cap, 0);
    HIP_TRY(hipMemcpyAsync(rn.data(), K.rnorm, sizeof(double) * cap, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(bn.data(), K.bnorm, sizeof(double) * cap, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(mind.data(), min_den, sizeof(double) * cap, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(flags.data(), K.flags, sizeof(int) * cap, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    rel.assign(cap, 0.0);
    for (int i = 0; i < cap; ++i) rel[i] = bn[i] > 0 ? rn[i] / bn[i] : 0.0;
    return FM_OK;
}

void set_error(const std::string &msg) { g_err = msg; }

std::recursive_mutex &hip_setup_mutex() {
    static std::recursive_mutex m;
    return m;
}

std::string upload(fm_problem *p, const HostFactors &hf) {
    std::string err;
    ProblemDev &pd = p->pd;
    pd.tile_lds = 0;
    pd.plane_lds = 0;
    pd.group_lds = 0;
    std::vector<int> gtile;              // grouped operator tiles (GT_REC ints each)
    pd.nodes_total = 0;
    for (int a = 0; a < 3; ++a) pd.nodes_total += 3 + p->bx[a].K + p->by[a].K + p->bz[a].K;
    pd.q[0] = p->bx[0].q;
    pd.q[1] = p->by[0].q;
    pd.q[2] = p->bz[0].q;
    for (int a = 1; a < 3; ++a) {
        if (p->bx[a].q != pd.q[0]) pd.q[0] = 0;
        if (p->by[a].q != pd.q[1]) pd.q[1] = 0;
        if (p->bz[a].q != pd.q[2]) pd.q[2] = 0;
    }
    for (int a = 0; a < 3; ++a) {
        CompDev &C = pd.comp[a];
        C.x = dim_dev(p, p->bx[a], err);
        C.y = dim_dev(p, p->by[a], err);
        C.z = dim_dev(p, p->bz[a], err);
        C.off = p->off[a];
        C.nxy = p->bx[a].n * p->by[a].n;
        C.npts = int(p->npts[a]);
        C.P = put(p, hf.comp[a].P, err);
        C.Vs = put(p, hf.comp[a].Vs, err);
        for (int b = 0; b < 3; ++b) {
            C.c[b] = p->crot[b][a];
            C.s[b] = p->srot[b][a];
        }
        C.xt = std::max(1, 256 / p->by[a].n);
        C.xt = std::min(C.xt, p->bx[a].n);
        C.ntiles = p->bz[a].n * ((p->bx[a].n + C.xt - 1) / C.xt);
        // LDS of the operator kernels: three z-contracted planes over
        // (x support of xt consecutive points, or of gt x groups) x ny
        {
            const Basis1D &bz = p->bz[a], &bx = p->bx[a];
            int rx = 0;
            for (int i0 = 0; i0 < bx.n; i0 += C.xt) {
                int lo = 1 << 30, hi = -1;
                for (int i = i0; i < std::min(bx.n, i0 + C.xt); ++i)
                    for (int s = 0; s < MAXR; ++s) {
                        int g = bx.idx[size_t(i) * MAXR + s];
                        if (g >= 0) { lo = std::min(lo, g); hi = std::max(hi, g); }
                    }
                rx = std::max(rx, hi - lo + 1);
            }
            pd.plane_lds = std::max(pd.plane_lds, 3 * rx * p->by[a].n);
            // x groups and the grouped tiles (three planes plus the x rows of the tile's points)
            std::vector<int> xg;
            for (int i = 0; i < bx.n; ++i) {
                const bool same = i > 0 && int(i - xg.back()) < 4 &&
                                  std::equal(bx.idx.begin() + size_t(i) * MAXR, bx.idx.begin() + size_t(i + 1) * MAXR,
                                             bx.idx.begin() + size_t(i - 1) * MAXR);
                if (!same) xg.push_back(i);
            }
            C.ngx = int(xg.size());
            xg.push_back(bx.n);
            C.gt = std::max(1, std::min(C.ngx, 256 / p->by[a].n));
            C.ntiles_g = bz.n * ((C.ngx + C.gt - 1) / C.gt);
            for (int g0 = 0; g0 < C.ngx; g0 += C.gt) {
                const int i0 = xg[g0], i1 = xg[std::min(C.ngx, g0 + C.gt)];
                int lo = 1 << 30, hi = -1;
                for (int i = i0; i < i1; ++i)
                    for (int s = 0; s < MAXR; ++s) {
                        int g = bx.idx[size_t(i) * MAXR + s];
                        if (g >= 0) { lo = std::min(lo, g); hi = std::max(hi, g); }
                    }
                pd.group_lds = std::max(pd.group_lds, 3 * (hi - lo + 1) * p->by[a].n + (i1 - i0) * 2 * MAXR);
            }
            C.xg = put(p, xg, err);
            // the tiles' records, in the order the kernel's blocks take them
            const int ntg = (C.ngx + C.gt - 1) / C.gt;
            for (int iz = 0; iz < bz.n && !p->absent(a); ++iz)
                for (int tg = 0; tg < ntg; ++tg) {
                    const int g0 = tg * C.gt, ngt = std::min(C.gt, C.ngx - g0);
                    const int ixs = xg[g0], ixe = xg[g0 + ngt];
                    int lo = 1 << 30, hi = -1;
                    for (int i = ixs; i < ixe; ++i)
                        for (int s = 0; s < MAXR; ++s) {
                            int g = bx.idx[size_t(i) * MAXR + s];
                            if (g >= 0) { lo = std::min(lo, g); hi = std::max(hi, g); }
                        }
                    const int rec[GT_REC] = {a, iz, g0, ngt, ixs, ixe, lo, hi};
                    gtile.insert(gtile.end(), rec, rec + GT_REC);
                }
        }
        PrecCompDev &F = p->pr.comp[a];
        std::memset(&F, 0, sizeof(F));
        if (p->absent(a)) {
            // implied by component 1 (exchange symmetry): no points, slices or tiles
            C.npts = 0;
            C.nxy = 0;
            C.z.n = 0;
            C.ntiles = C.ntiles_g = 0;
            continue;
        }
        F.nx = p->bx[a].n;
        F.ny = p->by[a].n;
        F.nz = p->bz[a].n;
        F.nM = p->nM;
        const HostComp &h = hf.comp[a];
        F.Wz = put(p, h.Wz, err);
        F.Wx = put(p, h.Wx, err);
        F.Wy = put(p, h.Wy, err);
        F.lx = put(p, h.lx, err);
        F.lxi = put(p, h.lxi, err);
        F.ly = put(p, h.ly, err);
        F.lyi = put(p, h.lyi, err);
        F.tx = put(p, h.tx, err);
        F.ty = put(p, h.ty, err);
        // FP32 copies and bfloat16 (hi, mid) planes of the factors
        auto to32 = [](const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); };
        auto to16 = [](const std::vector<double> &v) {
            std::vector<unsigned short> o(2 * v.size());
            for (size_t i = 0; i < v.size(); ++i) {
                float f = float(v[i]);
                unsigned short hi = bf16_rne(f);
                o[i] = hi;
                o[v.size() + i] = bf16_rne(f - bf16_value(hi));
            }
            return o;
        };
        F.Wz32 = put(p, to32(h.Wz), err);
        F.Wx32 = put(p, to32(h.Wx), err);
        F.Wy32 = put(p, to32(h.Wy), err);
        F.Wx16 = put(p, to16(h.Wx), err);
        F.Wy16 = put(p, to16(h.Wy), err);
        if (p->variant == 2) F.Zj = put(p, h.Zj, err);
        if (!err.empty()) return err;
    }
    p->pr.coupled = p->variant == 2 ? 1 : 0;
    {
        // the slices with complex pencil pairs, in the kernels' slice numbering
        std::vector<int> ps;
        int base = 0;
        for (int a = 0; a < 3; ++a) {
            if (p->absent(a)) continue;
            const HostComp &h = hf.comp[a];
            const int nx = p->bx[a].n, ny = p->by[a].n, ns = p->nM * p->bz[a].n;
            for (int sl = 0; sl < ns; ++sl) {
                bool any = false;
                for (int i = 0; i < nx && !any; ++i) any = h.tx[size_t(sl) * nx + i] != 0;
                for (int j = 0; j < ny && !any; ++j) any = h.ty[size_t(sl) * ny + j] != 0;
                if (any) ps.push_back(base + sl);
            }
            base += ns;
        }
        p->pr.npair_slices = int(ps.size());
        p->pr.pair_slices = put(p, ps, err);
    }
    pd.gtile = put(p, gtile, err);
    if (!err.empty()) return err;
    pd.tile_lds = std::max(pd.plane_lds, pd.group_lds);
    // coupling pairs for the tiled operator
    pd.cpl = CouplingDev{};
    if (sizeof(double) * size_t(pd.tile_lds) > 64 * 1024 && matvec_tiled_ok(pd))
        prepare_operator_lds(sizeof(double) * size_t(pd.tile_lds));
    if (p->exchange != 0 && !matvec_tiled_ok(pd))
        return "invalid: exchange-reduced problems need the tiled operator (one spline order in x, y and in z, "
               "2q <= n_y <= 256)";
    if (matvec_tiled_ok(pd)) {
        if (2 * p->N >= (1LL << 31)) return "problem too large for the tiled operator";
        CouplingHost ch;
        err = build_coupling(p, hf, ch);
        if (!err.empty()) return err;
        pd.cpl.ntasks = ch.ntasks;
        pd.cpl.njobs = ch.njobs;
        pd.cpl.pairs_per_lane = ch.pairs_per_lane;
        pd.cpl.jrec = put(p, ch.jrec, err);
        pd.cpl.npairs = ch.npairs;
        // with one M'' block the kernels read the job-ordered copies only
        pd.cpl.task = p->nM == 1 ? nullptr : put(p, ch.task, err);
        pd.cpl.r = put(p, ch.r, err);
        pd.cpl.out = put(p, ch.out, err);
        pd.cpl.s = put(p, ch.s, err);
        pd.cpl.F = put(p, ch.F, err);
        if (!err.empty()) return err;
    }
    // device copies of the two descriptors
    pd.dev = nullptr;
    p->pr.dev = nullptr;
    std::vector<ProblemDev> pdv(1, pd);
    std::vector<PrecDev> prv(1, p->pr);
    pd.dev = put(p, pdv, err);
    p->pr.dev = put(p, prv, err);
    return err;
}

}  // namespace fm

using namespace fm;

extern "C" {

const char *fm_last_error(void) { return g_err.c_str(); }

fm_status fm_create_problem(const fm_problem_desc *desc, fm_problem **out) {
    if (!desc || !out) return fail(FM_E_INVALID, "null argument");
    fm_problem *p = new (std::nothrow) fm_problem();
    if (!p) return fail(FM_E_NOMEM, "host allocation failed");
    p->desc = *desc;
    std::string e = setup_problem(p);
    if (!e.empty()) {
        delete p;
        return fail(FM_E_INVALID, e);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || desc->device < 0 || desc->device >= ndev) {
        delete p;
        return fail(FM_E_HIP, "no such HIP device");
    }
    if (hipSetDevice(desc->device) != hipSuccess) {
        delete p;
        return fail(FM_E_HIP, "hipSetDevice failed");
    }
    // LDS per block: the fused x-y kernels (slices of side <= 32) and the tiled
    // operator size their dynamic LDS from the problem; wider slices run as
    // batched GEMMs with fixed tiles
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, desc->device) != hipSuccess) {
            delete p;
            return fail(FM_E_HIP, "cannot query LDS size");
        }
        p->pd.lds_max = lds;
        for (int a = 0; a < 3; ++a) {
            size_t padded = sizeof(double) * size_t((p->bx[a].n + 15) & ~15) * (((p->by[a].n + 15) & ~15) + 4);
            if (p->bx[a].n <= XY_FUSED_MAX_SIDE && p->by[a].n <= XY_FUSED_MAX_SIDE && padded <= size_t(lds))
                prepare_large_lds(padded);
        }
    }
    HostFactors hf;
    e = build_factors(p, hf);
    if (!e.empty()) {
        delete p;
        return fail(FM_E_PENCIL, e);
    }
    p->pencil_err = hf.max_err;
    {
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        e = upload(p, hf);
    }
    if (!e.empty()) {
        fm_destroy_problem(p);
        const bool invalid = e.rfind("invalid: ", 0) == 0;
        return fail(invalid ? FM_E_INVALID : FM_E_NOMEM, invalid ? e.substr(9) : e);
    }
    *out = p;
    return FM_OK;
}

fm_status fm_destroy_problem(fm_problem *p) {
    if (!p) return FM_OK;
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    (void)hipSetDevice(p->desc.device);
    for (auto &b : p->buffers) (void)hipFree(b.ptr);
    if (p->ws) (void)hipFree(p->ws);
    if (p->ws_small) (void)hipFree(p->ws_small);
    if (p->cbuf) (void)hipFree(p->cbuf);
    if (p->ptmp) (void)hipFree(p->ptmp);
    if (p->host_pinned) (void)hipHostFree(p->host_pinned);
    for (auto e : p->prof.ev) (void)hipEventDestroy(e);
    if (p->solve_batch) {
        p->solve_batch->release();
        delete p->solve_batch;
    }
    delete p;
    return FM_OK;
}

fm_status fm_problem_info(const fm_problem *p, size_t *n_unknowns, size_t *bytes_resident, int restart,
                          size_t *bytes_per_request) {
    if (!p) return fail(FM_E_INVALID, "null problem");
    if (n_unknowns) *n_unknowns = size_t(p->N);
    if (bytes_resident) *bytes_resident = p->bytes_resident;
    if (bytes_per_request) {
        if (restart < 1) return fail(FM_E_INVALID, "restart must be >= 1");
        *bytes_per_request = krylov_bytes(p->N, 1, restart);
    }
    return FM_OK;
}

fm_status fm_apply_operator(fm_problem *p, int nbatch, const double *E, const double *x_dev, double *y_dev,
                            void *stream) {
    if (!p || !E || !x_dev || !y_dev || nbatch < 1) return fail(FM_E_INVALID, "bad argument");
    if (x_dev == y_dev) return fail(FM_E_INVALID, "x and y must not overlap");
    Busy busy(p);
    if (!busy.ok) return fail(FM_E_BUSY, "problem handle in use");
    HIP_TRY(hipSetDevice(p->desc.device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Small s;
    fm_status r = ensure_small(p, nbatch, s);
    if (r != FM_OK) return r;
    HIP_TRY(hipMemcpyAsync(s.E, E, sizeof(double) * nbatch, hipMemcpyHostToDevice, st));
    const size_t cb = sizeof(double) * 2 * size_t(nbatch) * size_t(p->N);
    if (p->cbuf_bytes < cb) {
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        if (p->cbuf) (void)hipFree(p->cbuf);
        p->cbuf = nullptr;
        p->cbuf_bytes = 0;
        HIP_TRY(hipMalloc(&p->cbuf, cb));
        p->cbuf_bytes = cb;
        HIP_TRY(hipMemsetAsync(p->cbuf, 0, cb, st));
    }
    apply_operator(p, nbatch, s.E, nullptr, x_dev, y_dev, p->cbuf, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    add_matvec_work(p, Work(p), nbatch);
    prof_collect(p);
    return FM_OK;
}

fm_status fm_apply_precond(fm_problem *p, int nbatch, const double *E, const double *r_dev, double *z_dev, int prec,
                           void *stream) {
    if (!p || !E || !r_dev || !z_dev || nbatch < 1) return fail(FM_E_INVALID, "bad argument");
    if (prec != FM_FP64 && prec != FM_FP32 && prec != FM_BF16X3) return fail(FM_E_INVALID, "bad precision");
    Busy busy(p);
    if (!busy.ok) return fail(FM_E_BUSY, "problem handle in use");
    HIP_TRY(hipSetDevice(p->desc.device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Small s;
    fm_status r = ensure_small(p, nbatch, s);
    if (r != FM_OK) return r;
    HIP_TRY(hipMemcpyAsync(s.E, E, sizeof(double) * nbatch, hipMemcpyHostToDevice, st));
    const size_t tb = sizeof(double) * size_t(nbatch) * size_t(p->N);
    if (p->ptmp_bytes < tb) {
        std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
        if (p->ptmp) (void)hipFree(p->ptmp);
        p->ptmp = nullptr;
        p->ptmp_bytes = 0;
        HIP_TRY(hipMalloc(&p->ptmp, tb));
        p->ptmp_bytes = tb;
    }
    apply_precond(p, nbatch, s.E, nullptr, r_dev, z_dev, prec, nullptr, p->ptmp, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    add_precond_work(p, Work(p), nbatch);
    prof_collect(p);
    return FM_OK;
}

fm_status fm_solve(fm_problem *p, int nbatch, const double *E, const double *b_dev, double *x_dev,
                   const fm_solve_opts *opts, fm_solve_result *results, void *stream) {
    if (!p || !E || !b_dev || !x_dev || !opts || nbatch < 1) return fail(FM_E_INVALID, "bad argument");
    const int m = opts->restart;
    if (m < 1 || m > MAX_RESTART) return fail(FM_E_INVALID, "restart must be in [1, 1000]");
    if (!(opts->rtol > 0)) return fail(FM_E_INVALID, "rtol must be positive");
    if (opts->max_iters < 1) return fail(FM_E_INVALID, "max_iters must be >= 1");
    if (opts->prec != FM_FP64 && opts->prec != FM_FP32 && opts->prec != FM_BF16X3)
        return fail(FM_E_INVALID, "bad precision");
    for (int i = 0; i < nbatch; ++i)
        if (!std::isfinite(E[i])) return fail(FM_E_INVALID, "non-finite energy");
    Busy busy(p);
    if (!busy.ok) return fail(FM_E_BUSY, "problem handle in use");
    HIP_TRY(hipSetDevice(p->desc.device));
    return solve_locked(p, nbatch, E, b_dev, x_dev, opts, results, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace fm {
namespace {
// Device energies of nbc complex requests: Re E per row (2 nbc), Re E and
// Im E per request (nbc each), in the problem's small workspace.
fm_status complex_energies(fm_problem *p, int nbc, const double *E_re, const double *E_im, hipStream_t st,
                           double **E2, double **Ere, double **Eim) {
    Small s;
    fm_status r = ensure_small(p, 2 * nbc, s);     // s.E: 2 nbc doubles, s.min_den: 2 nbc doubles
    if (r != FM_OK) return r;
    std::vector<double> e2(2 * size_t(nbc)), ri(2 * size_t(nbc));
    for (int c = 0; c < nbc; ++c) {
        e2[2 * c] = e2[2 * c + 1] = E_re[c];
        ri[c] = E_re[c];
        ri[nbc + c] = E_im[c];
    }
    HIP_TRY(hipMemcpyAsync(s.E, e2.data(), sizeof(double) * 2 * nbc, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s.min_den, ri.data(), sizeof(double) * 2 * nbc, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    *E2 = s.E;
    *Ere = s.min_den;
    *Eim = s.min_den + nbc;
    return FM_OK;
}

fm_status grow(fm_problem *p, double *&buf, size_t &have, size_t bytes, bool zero, hipStream_t st) {
    if (have >= bytes) return FM_OK;
    std::lock_guard<std::recursive_mutex> lock(hip_setup_mutex());
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    have = 0;
    HIP_TRY(hipMalloc(&buf, bytes));
    have = bytes;
    if (zero) HIP_TRY(hipMemsetAsync(buf, 0, bytes, st));
    return FM_OK;
}

bool energies_finite(int n, const double *a, const double *b) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(a[i]) || !std::isfinite(b[i])) return false;
    return true;
}
}  // namespace
}  // namespace fm

extern "C" {

fm_status fm_apply_operator_complex(fm_problem *p, int nbatch, const double *E_re, const double *E_im,
                                    const double *x_dev, double *y_dev, void *stream) {
    if (!p || !E_re || !E_im || !x_dev || !y_dev || nbatch < 1) return fail(FM_E_INVALID, "bad argument");
    if (x_dev == y_dev) return fail(FM_E_INVALID, "x and y must not overlap");
    if (!energies_finite(nbatch, E_re, E_im)) return fail(FM_E_INVALID, "non-finite energy");
    Busy busy(p);
    if (!busy.ok) return fail(FM_E_BUSY, "problem handle in use");
    HIP_TRY(hipSetDevice(p->desc.device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *E2, *Ere, *Eim;
    fm_status r = complex_energies(p, nbatch, E_re, E_im, st, &E2, &Ere, &Eim);
    if (r != FM_OK) return r;
    const size_t rows = 2 * size_t(nbatch);
    r = grow(p, p->cbuf, p->cbuf_bytes, sizeof(double) * 2 * rows * size_t(p->N), true, st);
    if (r != FM_OK) return r;
    r = grow(p, p->ptmp, p->ptmp_bytes, sizeof(double) * rows * size_t(p->N), false, st);
    if (r != FM_OK) return r;
    apply_operator_complex(p, nbatch, E2, Eim, nullptr, nullptr, x_dev, y_dev, p->cbuf, p->ptmp, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    prof_collect(p);
    return FM_OK;
}

fm_status fm_apply_precond_complex(fm_problem *p, int nbatch, const double *E_re, const double *E_im,
                                   const double *r_dev, double *z_dev, void *stream) {
    if (!p || !E_re || !E_im || !r_dev || !z_dev || nbatch < 1) return fail(FM_E_INVALID, "bad argument");
    if (!energies_finite(nbatch, E_re, E_im)) return fail(FM_E_INVALID, "non-finite energy");
    Busy busy(p);
    if (!busy.ok) return fail(FM_E_BUSY, "problem handle in use");
    HIP_TRY(hipSetDevice(p->desc.device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *E2, *Ere, *Eim;
    fm_status r = complex_energies(p, nbatch, E_re, E_im, st, &E2, &Ere, &Eim);
    if (r != FM_OK) return r;
    r = grow(p, p->ptmp, p->ptmp_bytes, sizeof(double) * 2 * size_t(nbatch) * size_t(p->N), false, st);
    if (r != FM_OK) return r;
    apply_precond_complex(p, nbatch, Ere, Eim, nullptr, nullptr, r_dev, z_dev, nullptr, p->ptmp, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    prof_collect(p);
    return FM_OK;
}

fm_status fm_solve_complex(fm_problem *p, int nbatch, const double *E_re, const double *E_im, const double *b_dev,
                           double *x_dev, const fm_solve_opts *opts, fm_solve_result *results, void *stream) {
    if (!p || !E_re || !E_im || !b_dev || !x_dev || !opts || nbatch < 1) return fail(FM_E_INVALID, "bad argument");
    const int m = opts->restart;
    if (m < 1 || m > MAX_RESTART) return fail(FM_E_INVALID, "restart must be in [1, 1000]");
    if (!(opts->rtol > 0)) return fail(FM_E_INVALID, "rtol must be positive");
    if (opts->max_iters < 1) return fail(FM_E_INVALID, "max_iters must be >= 1");
    if (opts->prec != FM_FP64) return fail(FM_E_INVALID, "complex energies run FP64 products only");
    if (!energies_finite(nbatch, E_re, E_im)) return fail(FM_E_INVALID, "non-finite energy");
    Busy busy(p);
    if (!busy.ok) return fail(FM_E_BUSY, "problem handle in use");
    HIP_TRY(hipSetDevice(p->desc.device));
    return solve_locked(p, nbatch, E_re, b_dev, x_dev, opts, results, static_cast<hipStream_t>(stream), E_im);
}

fm_status fm_apply_mass(fm_problem *p, int nbatch, const double *x_dev, double *y_dev, void *stream) {
    if (!p || !x_dev || !y_dev || nbatch < 1) return fail(FM_E_INVALID, "bad argument");
    if (x_dev == y_dev) return fail(FM_E_INVALID, "x and y must not overlap");
    Busy busy(p);
    if (!busy.ok) return fail(FM_E_BUSY, "problem handle in use");
    HIP_TRY(hipSetDevice(p->desc.device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_mass(p->pd, nbatch, x_dev, y_dev, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return FM_OK;
}

}  // extern "C"

namespace fm {

// fm_solve after validation, with the handle held and the device set.
fm_status solve_locked(fm_problem *p, int nbatch, const double *E, const double *b_dev, double *x_dev,
                       const fm_solve_opts *opts, fm_solve_result *results, hipStream_t st, const double *E_im) {
    const int m = opts->restart;
    const int cplx = E_im ? 1 : 0;
    // the problem keeps the batch of its last solve for reuse
    Batch *b = p->solve_batch;
    if (!b || b->cap != nbatch || b->m != m || b->cplx != cplx) {
        if (b) {
            b->release();
            delete b;
            p->solve_batch = nullptr;
        }
        b = new (std::nothrow) Batch();
        if (!b) return fail(FM_E_NOMEM, "host allocation failed");
        fm_status r = b->create(p, nbatch, m, st, cplx);
        if (r != FM_OK) {
            delete b;
            return r;
        }
        p->solve_batch = b;
    }
    b->st = st;
    b->B = b_dev;
    b->X = x_dev;
    b->prec = opts->prec;
    b->graphs = opts->graphs;
    b->rtol = opts->rtol;
    std::vector<int> all(nbatch);
    for (int i = 0; i < nbatch; ++i) {
        all[i] = i;
        b->E[i] = E[i];
        if (cplx) b->Ei[i] = E_im[i];
        b->limit[i] = opts->max_iters;
    }
    fm_status r = b->boundary(all, opts->x0_is_guess);
    if (r != FM_OK) return r;
    int guard = 0;
    while (b->any_running() && ++guard < 1000000) {
        r = b->cycle(nullptr, 0);
        if (r != FM_OK) return r;
        r = b->boundary({}, opts->x0_is_guess);
        if (r != FM_OK) return r;
    }
    std::vector<double> rel, md;
    std::vector<int> fl;
    r = b->read_results(rel, md, fl);
    if (r != FM_OK) return r;
    fm_status overall = FM_OK;
    for (int i = 0; i < nbatch; ++i) {
        int stt = FM_OK;
        if (fl[i] & 1) stt = FM_E_NONFINITE;
        else if (fl[i] & 2) stt = FM_E_NONFINITE;
        else if (!(rel[i] <= opts->rtol)) stt = FM_E_NOT_CONVERGED;
        if (stt != FM_OK && (overall == FM_OK || stt == FM_E_NONFINITE)) overall = (fm_status)stt;
        if (results) {
            results[i].iters = b->iters[i];
            results[i].restarts = b->restarts[i];
            results[i].rel_residual = rel[i];
            results[i].min_abs_denominator = md[i];
            results[i].status = stt;
        }
    }
    if (overall == FM_E_NOT_CONVERGED) g_err = "some requests did not reach rtol";
    if (overall == FM_E_NONFINITE) g_err = "non-finite value in b or during the iteration";
    return overall;
}

}  // namespace fm

extern "C" {

fm_status fm_profile(fm_problem *p, int enable) {
    if (!p) return fail(FM_E_INVALID, "null problem");
    Profile &pf = p->prof;
    pf.on = enable != 0;
    pf.recs.clear();
    pf.next = 0;
    for (int c = 0; c < FM_K_COUNT; ++c) {
        pf.ms[c] = 0;
        pf.launches[c] = 0;
        pf.bytes[c] = 0;
        pf.flops[c] = 0;
    }
    return FM_OK;
}

fm_status fm_profile_read(const fm_problem *p, int kclass, double *total_ms, long long *launches, double *bytes,
                          double *flops) {
    if (!p || kclass < 0 || kclass >= FM_K_COUNT) return fail(FM_E_INVALID, "bad argument");
    const Profile &pf = p->prof;
    if (total_ms) *total_ms = pf.ms[kclass];
    if (launches) *launches = pf.launches[kclass];
    if (bytes) *bytes = pf.bytes[kclass];
    if (flops) *flops = pf.flops[kclass];
    return FM_OK;
}

}  // extern "C"

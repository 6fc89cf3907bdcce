// The problem handle and host-side factor storage.
#pragma once

#include <mutex>

#include "fm_internal.h"

namespace fm {

struct HostComp {
    std::vector<double> Wz, Wx, Wy, lx, lxi, ly, lyi, P, Vs;
    std::vector<double> Zj;      // coupled variant: joint z matrices [2][nM nz][nM nz]
    std::vector<signed char> tx, ty;
};

struct HostFactors {
    HostComp comp[3];
    double max_err = 0;
};

struct CouplingHost {
    std::vector<int> task, out;  // task: [ntasks][CPL_TASK] records
    std::vector<int> job;        // [njobs][2] wave jobs (second task -1 for a single one)
    std::vector<int> jrec;       // one M'' block: [njobs][2][CPL_TASK] job-ordered records (CouplingDev::jrec)
    int njobs = 0;
    int pairs_per_lane = 1;
    std::vector<double> s, F, r; // r: [ntasks][3] cell width / hbar (z, x, y)
    long long npairs = 0;
    int ntasks = 0;
};

struct Profile {
    bool on = false;
    std::vector<hipEvent_t> ev;
    size_t next = 0;
    struct Rec {
        int cls;
        size_t e0, e1;
    };
    std::vector<Rec> recs;
    double ms[FM_K_COUNT] = {0};
    long long launches[FM_K_COUNT] = {0};
    double bytes[FM_K_COUNT] = {0};
    double flops[FM_K_COUNT] = {0};
};

struct Batch;

struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace fm

struct fm_problem {
    fm_problem_desc desc;
    int nM = 0, M0 = 0;
    int variant = 1;                         // preconditioner: 1 block-Jacobi in M', 2 coupled
    double mode_fit_tol = FM_DEFAULT_MODE_FIT_TOL;   // coupled: z modes fitting g_l^{M'} within this
    int exchange = 0;                        // +-1: component 2 (index 1) is implied by component 1 (index 0);
                                             // 3: components 2 and 3 are implied by component 1
    bool absent(int a) const { return exchange != 0 && (a == 1 || (exchange == 3 && a == 2)); }
    int zhalf = 0, zsigma = 1;               // component 3 on z in [0, 1] with parity zsigma
    long long N = 0;
    long long npts[3] = {0, 0, 0};
    long long off[3] = {0, 0, 0};
    double mu[3], mu_abc[3], zz[3];
    double crot[3][3], srot[3][3];
    fm::Basis1D bx[3], by[3], bz[3];
    fm::ProblemDev pd;
    fm::PrecDev pr;
    std::vector<fm::DeviceBuffer> buffers;   // factors, fields, basis tables
    size_t bytes_resident = 0;
    double pencil_err = 0;
    std::atomic<int> busy{0};
    // solver workspace (grown on demand)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *ws_small = nullptr;
    size_t ws_small_bytes = 0;
    double *cbuf = nullptr;                  // coupling buffer of fm_apply_operator ([nb][2][N], zeroed)
    size_t cbuf_bytes = 0;
    double *ptmp = nullptr;                  // scratch of fm_apply_precond ([nb][N])
    size_t ptmp_bytes = 0;
    double *host_pinned = nullptr;           // pinned host scratch for flag read-back
    size_t host_pinned_bytes = 0;
    fm::Profile prof;
    fm::Batch *solve_batch = nullptr;        // workspace of the last fm_solve, reused
};

namespace fm {
// Holds a problem handle for one call (one call at a time per handle).
struct Busy {
    fm_problem *p;
    bool ok;
    explicit Busy(fm_problem *q) : p(q) {
        int z = 0;
        ok = p->busy.compare_exchange_strong(z, 1);
    }
    ~Busy() {
        if (ok) p->busy.store(0);
    }
};
// fm_solve on a held handle with its device current (arguments already checked).
// E_im: imaginary parts of complex energies (nullptr: real energies); with
// them b_dev and x_dev hold [request][re, im][N].
fm_status solve_locked(fm_problem *p, int nbatch, const double *E, const double *b_dev, double *x_dev,
                       const fm_solve_opts *opts, fm_solve_result *results, hipStream_t st,
                       const double *E_im = nullptr);
std::string setup_problem(fm_problem *p);
std::string build_factors(fm_problem *p, HostFactors &hf);
std::string upload(fm_problem *p, const HostFactors &hf);
std::string build_coupling(const fm_problem *p, const HostFactors &hf, CouplingHost &ch);
// coupled preconditioner (coupled.cpp)
double assoc_g(int l, int M, double z);
std::string order_and_scale_z(const Basis1D &bz, int Mp, double fit_tol, std::vector<double> &Wb,
                              std::vector<double> &W, std::vector<double> &lre, std::vector<char> &resolved);
std::string coupled_slots(const fm_problem *p, int nz, const std::vector<std::vector<double>> &Wbz,
                          const std::vector<std::vector<double>> &Wz, const std::vector<std::vector<double>> &lz,
                          const std::vector<std::vector<char>> &resolved, std::vector<double> &Zj,
                          std::vector<double> &cx, std::vector<double> &cy);
void set_error(const std::string &msg);
// Serialises the library's own allocations, frees, stream creation and
// synchronous copies with its stream captures: while any stream of the process
// is being captured, HIP refuses synchronous calls on the null stream from
// every thread.  Recursive: a holder may call code that takes it again.
std::recursive_mutex &hip_setup_mutex();
}  // namespace fm

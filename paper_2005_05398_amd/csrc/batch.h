// A batch of flexible-GMRES solve slots of one problem sharing one Krylov
// workspace.  Every slot has its own energy, right-hand side (row of B) and
// solution (row of X); slots start at restart boundaries, so requests can join
// a batch that is already iterating.
#pragma once

#include <functional>

#include "fm_problem.h"

namespace fm {

struct Batch {
    fm_problem *p = nullptr;
    int cap = 0, m = 0;
    hipStream_t st = nullptr;
    KrylovDev K{};
    void *mem = nullptr;
    size_t bytes = 0;
    int *running = nullptr, *cont = nullptr, *fresh = nullptr;   // device masks [cap]
    double *min_den = nullptr;                                   // device [cap]
    double *cbuf = nullptr;                                      // device [cap][2][N] operator coupling
    double *ptmp = nullptr;                                      // device [cap][N] preconditioner scratch
    int *hbuf = nullptr;                                         // pinned host scratch [cap]
    const double *B = nullptr;                                   // [cap][N]
    double *X = nullptr;                                         // [cap][N]
    int prec = FM_FP64;
    double rtol = 1e-10;
    // Complex energies: every slot is a complex request, two rows (real and
    // imaginary part) of length N, so the Krylov vectors have length 2N.
    int cplx = 0;
    double *E2 = nullptr;                                        // device [2 cap]: Re E of each row
    double *Eim = nullptr;                                       // device [cap]: Im E
    int *mask2 = nullptr;                                        // device [2 cap]: row masks
    std::vector<double> Ei;                                      // host Im E per slot
    // Arnoldi steps run as replays of captured HIP graphs, one graph per group
    // of GRAPH_STEPS consecutive steps (per step index and precision, captured
    // on first use on a private stream and kept with the batch); eager
    // launches while per-launch profiling is on or if a capture fails.
    static constexpr int GRAPH_STEPS = 4;
    int graphs = 0;
    bool graphs_failed = false;
    hipStream_t cap_st = nullptr;
    std::vector<hipGraphExec_t> gexec;          // [prec][group]
    std::vector<int> run, iters, restarts, limit, last_steps;    // host view per slot
    std::vector<double> E;

    static size_t footprint(const fm_problem *p, int cap, int m, int cplx = 0);
    fm_status create(fm_problem *p, int cap, int m, hipStream_t st, int cplx = 0);
    void release();
    // Ends the cycle of the running slots (x += Z y, then the FP64 true
    // residual decides convergence) and starts the slots in `joining`, whose E
    // and B rows must already be set.  A slot over its step limit stops here.
    fm_status boundary(const std::vector<int> &joining, int x0_is_guess);
    // Stops running slots at a restart boundary (they leave the batch's
    // kernels; their X rows keep the last iterate).
    fm_status stop(const std::vector<int> &slots);
    // Arnoldi steps for the active slots until every slot stops, j reaches m,
    // or want_cut() holds after at least min_steps steps.
    fm_status cycle(const std::function<bool()> &want_cut, int min_steps);
    bool any_running() const;
    // Enqueues Arnoldi step j (preconditioner, operator, dot pass, finish,
    // update) on stream s; timed() wraps each launch only on the batch's own
    // stream when profiling.
    void enqueue_step(int j, hipStream_t s, bool profile);
    // The replayable graph of steps j0 .. j0 + n - 1 at the current precision
    // (nullptr if it cannot be captured).
    hipGraphExec_t step_graph(int j0, int n);
    // Per slot: relative true residual, min |denominator|, status flags.
    fm_status read_results(std::vector<double> &rel, std::vector<double> &min_abs_den, std::vector<int> &flags);
};

}  // namespace fm

/*
 * fm.h - C ABI of the MI355X Faddeev-Merkuriev spline-collocation solver.
 *
 * The library solves (H - E S) c = b, the collocation system of the 3D
 * Faddeev-Merkuriev equations in total-orbital-momentum representation
 * (Gradusov, Roudnev, Yarevsky, Yakovlev, arXiv:2005.05398, Sec. 3.1,
 * eq. (FM-pre) with the right-hand side moved to the left; H c = E S c), by
 * preconditioned flexible GMRES on one AMD gfx950 GPU.  The preconditioner is
 * the tensor-trick inverse of the separable left-hand operator of eq. (FM-fin)
 * (Sec. 3.2, eqs. (MDA), (prec-1), (prec-2)).
 *
 * Conventions for every entry point
 *   - Every call returns fm_status; nothing throws across the ABI.  On an
 *     error fm_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread).
 *   - Vectors are FP64, contiguous, in the order [request][alpha][M'][z][x][y]
 *     (y fastest; Sec. 3.2 orders the unknowns eta, xi, zeta).  "N" is the
 *     number of unknowns of one request, n_M * sum_alpha n_z n_x n_y
 *     (Sec. 3.1), n_M = J - M0 + 1, M0 = (1 - tau)/2.
 *   - Unknown vectors hold spline coefficients c (Sec. 3.1); right-hand
 *     sides and operator outputs live in collocation-row space (one value per
 *     collocation point, same ordering).
 *   - Pointers named *_dev are device pointers on the problem's device; the
 *     caller owns them.  The library owns its factors and workspaces.
 *   - stream is a hipStream_t passed as void* (NULL: the null stream).  Work
 *     is enqueued on it; calls return once enqueued, except fm_solve, which
 *     synchronises the stream at restart boundaries and before returning.
 *   - A problem handle serves one call at a time; a call that overlaps another
 *     on the same handle returns FM_E_BUSY.
 */
#ifndef FM_H
#define FM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FM_OK = 0,
    FM_E_INVALID = -1,        /* bad argument or problem description */
    FM_E_NOMEM = -2,          /* device or host allocation failed */
    FM_E_HIP = -3,            /* a HIP runtime call failed */
    FM_E_NOT_CONVERGED = -4,  /* max_iters reached; x holds the best iterate */
    FM_E_BREAKDOWN = -5,      /* GMRES breakdown that is not a lucky one */
    FM_E_PENCIL = -6,         /* a 1D pencil could not be diagonalised in real arithmetic */
    FM_E_NONFINITE = -7,      /* NaN or Inf in an input vector */
    FM_E_REJECTED = -8,       /* serving: request does not fit the memory budget */
    FM_E_BUSY = -9            /* handle already in use */
} fm_status;

typedef enum { FM_FP64 = 0, FM_FP32 = 1, FM_BF16X3 = 2 } fm_precision;

/* Spline node maps (Sec. 4): x, y use UNIFORM, QUADRATIC (t_i = R (i/K)^2) or
 * POW (eq. (map-pow)); z uses SIN (sin(pi u / 2), u equidistant) or UNIFORM. */
typedef enum { FM_MAP_UNIFORM = 0, FM_MAP_QUADRATIC = 1, FM_MAP_POW = 2, FM_MAP_SIN = 3 } fm_map;

/* One 1D basis (Sec. 3.1, Sec. 4): Hermite splines of degree 3 (two functions
 * per node) or 5 (three functions per node, S_5^3) with Gauss collocation.
 *   x, y on [0, R] with zero Dirichlet conditions at both ends:
 *        degree 3: n = 2K;  degree 5: n = 3K + 1.
 *   z on [-1, 1] (R ignored): degree 3: n = 2K + 2, n >= 4;
 *        degree 5: n = 3K + 3, n >= 6.
 * K is the number of intervals. */
typedef struct {
    int degree;
    int n;
    double R;
    int map;                  /* fm_map */
} fm_dim;

/* The problem statement (Sec. 2.1-2.2): masses and charges of the three
 * particles, total orbital momentum J and parity tau, one basis triple per
 * Faddeev component, the Merkuriev cut-off of eq. (Mcutoff0) (y0 may be
 * +INFINITY) and the choice of Vhat of eq. (FM-fin) (0: Z_a (Z_b + Z_c)
 * sqrt(2 mu_a(bc)) / (y + 1), Sec. 3.1), and the preconditioner variant
 * (FM_PREC_BLOCK_JACOBI or FM_PREC_COUPLED, see fm_apply_precond; 0 selects
 * the block-Jacobi one).  The energy is not part of it: all device-resident
 * factors are independent of E. */
typedef enum { FM_PREC_BLOCK_JACOBI = 1, FM_PREC_COUPLED = 2 } fm_prec_variant;

typedef struct {
    double mass[3];
    double charge[3];
    int J;                    /* total orbital momentum, 0 <= J <= 15 (n_M = J - M0 + 1 <= 16 blocks) */
    int tau;                  /* +1 or -1 */
    fm_dim x[3], y[3], z[3];  /* per component alpha */
    double x0, y0, nu;
    int vhat;
    int device;               /* HIP device ordinal */
    int precond;              /* fm_prec_variant (0: FM_PREC_BLOCK_JACOBI) */
    int exchange;             /* 0: all three components.  +1 / -1: particles 1 and 2 are identical
                                 (equal masses, charges and component bases) and only the part of
                                 parity p = exchange under their permutation is solved: components 1
                                 and 3 (Sec. 2, "Permutational symmetry", eq. (2-sym-part): component
                                 2 is p (-1)^{M'} times component 1 at -z); vectors then hold
                                 [alpha = 1, 3][M'][z][x][y] and N = n_M (n_1 + n_3).
                                 3: all three particles are identical (equal masses, charges and
                                 component bases): psi_1 = psi_2 = psi_3 in their own coordinates
                                 (eq. (3-sym-part)) and only component 1 is solved, its coupling
                                 reading component 1 at both partners' rotated points; vectors hold
                                 [M'][z][x][y] of component 1 and N = n_M n_1.  Both parities of the
                                 full permutations are held (they are the parts of psi_1 even and odd
                                 under psi(x, y, z) -> (-1)^{M'} psi(x, y, -z)) */
    int zhalf;                /* 0: every component on z in [-1, 1].  1 (with exchange = +-1 and n_M = 1):
                                 component 3, symmetric or antisymmetric in z (parity
                                 sigma = p (-1)^{M0}, eq. (2-sym-part)), is solved on z in [0, 1]: its
                                 z basis is the part of the basis z[2] (which needs an even number of
                                 intervals, so that z = 0 is a node) on [0, 1], with the functions at
                                 z = 0 restricted to the parity, and its collocation points those of
                                 z[2] in [0, 1] (z = 0 itself only for an even quintic basis); the
                                 coupling reads it at |z_3| times sigma for z_3 < 0.  Its n_z becomes
                                 n/2 (cubic), 3K/2 + 2 (quintic, sigma = +1) or 3K/2 + 1 (quintic,
                                 sigma = -1) for n = 3K + 3 */
    double mode_fit_tol;      /* coupled preconditioner only (Sec. 3.2, eq. (prop-eq)): a z mode (M', k)
                                 whose computed eigenvector matches g_{M'+k}^{M'} at the collocation
                                 points with a relative least-squares residual above this keeps its
                                 computed eigenvalue and has no M' +- 1 coupling (the block-Jacobi
                                 treatment of that mode); the substitution of eq. (prop-eq) is made for
                                 the others.  <= 0: FM_DEFAULT_MODE_FIT_TOL; >= 1: every mode (the
                                 paper's matrix as printed) */
} fm_problem_desc;

#define FM_DEFAULT_MODE_FIT_TOL 0.02

typedef struct fm_problem fm_problem;

typedef struct {
    int restart;              /* Krylov space size m per cycle (>= 1) */
    double rtol;              /* stop when ||b - A x||_2 <= rtol ||b||_2 (true FP64 residual) */
    int max_iters;            /* total Arnoldi steps per request, checked at restart boundaries (a request
                                 stops at the first boundary at or past it, so it may take up to
                                 restart - 1 steps more) */
    int prec;                 /* fm_precision of the preconditioner's products */
    int x0_is_guess;          /* 1: x_dev holds the initial guess; 0: start from x = 0 */
    int graphs;               /* 1: the Arnoldi steps run as replays of HIP graphs captured on first use
                                 (four steps per graph, kept with the problem's workspace); 0: launched
                                 one kernel at a time.  Results are the same either way */
} fm_solve_opts;

typedef struct {
    int iters;                /* Arnoldi steps taken */
    int restarts;             /* completed cycles */
    double rel_residual;      /* final ||b - A x|| / ||b||, FP64 */
    double min_abs_denominator; /* min |lambda_x + lambda_y - E| over the divide */
    int status;               /* fm_status of this request */
} fm_solve_result;

/* Thread-local message of the last failing call on this thread. */
const char *fm_last_error(void);

/* Build all energy-independent data of a problem on the host in FP64 (1D
 * bases, the z, x and y pencils of Sec. 3.2 and their generalized
 * eigendecompositions (W-bar, W, Lambda) = D(A1, A2) of eq. (WW-scale),
 * potential fields) and upload it to the device.  Complex-conjugate
 * eigenvalue pairs of the x and y pencils are kept as real 2x2 blocks.
 * Errors: FM_E_INVALID (bad description; an exchange-reduced description
 * also needs one spline order in x and y and one in z over the components
 * and 2q <= n_y <= 256), FM_E_PENCIL (a z pencil with a complex
 * spectrum, or a diagonalisation that fails its accuracy check), FM_E_NOMEM,
 * FM_E_HIP.  *out is set only on FM_OK. */
fm_status fm_create_problem(const fm_problem_desc *desc, fm_problem **out);

/* Free a problem and its device memory.  NULL is accepted. */
fm_status fm_destroy_problem(fm_problem *p);

/* n_unknowns: N of one request.  bytes_resident: device bytes held by the
 * problem (factors and fields).  bytes_per_request(restart): device bytes of
 * the Krylov workspace one request needs at that restart length.
 * Any output pointer may be NULL. */
fm_status fm_problem_info(const fm_problem *p, size_t *n_unknowns, size_t *bytes_resident,
                          int restart, size_t *bytes_per_request);

/* y = (H - E S) x for nbatch requests at once (Sec. 3.1): the collocation
 * operator of eq. (FM-pre) with its coupling sum moved to the left.
 * E: host array of nbatch energies.  x_dev, y_dev: nbatch * N doubles each;
 * they must not overlap.  Errors: FM_E_INVALID, FM_E_HIP, FM_E_BUSY. */
fm_status fm_apply_operator(fm_problem *p, int nbatch, const double *E, const double *x_dev,
                            double *y_dev, void *stream);

/* z = L(E)^-1 r for nbatch requests, component by component (eq. (prec-1)).
 * FM_PREC_BLOCK_JACOBI: the tensor-trick inverse of the separable left-hand
 * operator of eq. (FM-fin) (Sec. 3.2) with the M' +- 1 blocks dropped
 * (block-Jacobi in M'; exact for n_M = 1).  FM_PREC_COUPLED: the inverse of
 * the paper's approximate matrix script-L of Sec. 3.2, which keeps the M' +- 1
 * blocks with the z eigenvalues replaced by -l(l+1) and the transformed
 * M' +- 1 blocks by the bidiagonal Lambda^{M'+-} (eq. (prop-eq); the z
 * eigenvectors ordered by |lambda| and scaled to the functions g_l^{M'} of
 * the Appendix).  prec selects the arithmetic of the x-y products (and, for
 * the block-Jacobi variant, of the z products); the divide by
 * lambda_x + lambda_y - E and the coupled variant's z products are always
 * FP64.  r_dev and z_dev may be the same buffer.  Errors: FM_E_INVALID,
 * FM_E_HIP, FM_E_BUSY. */
fm_status fm_apply_precond(fm_problem *p, int nbatch, const double *E, const double *r_dev,
                           double *z_dev, int prec, void *stream);

/* Solve (H - E_r S) x_r = b_r for nbatch requests that share the problem
 * (an energy scan), by right-preconditioned flexible GMRES(restart) with an
 * FP64 Arnoldi process that orthogonalises twice (classical Gram-Schmidt, the
 * second projection of each direction delayed to the next step so that one
 * step makes one pass of dot products and one pass of updates over the
 * basis), Givens rotations and an FP64 true residual at every restart (Sec. 4
 * names preconditioned GMRES as the linear solver of the method).  restart:
 * 1..1000.  Each request
 * stops on its own when its true residual meets rtol.  results: host array
 * of nbatch entries (may be NULL).  Returns FM_OK when every request
 * converged, FM_E_NOT_CONVERGED if any did not (x holds the last iterate),
 * FM_E_NONFINITE for a non-finite b. */
fm_status fm_solve(fm_problem *p, int nbatch, const double *E, const double *b_dev, double *x_dev,
                   const fm_solve_opts *opts, fm_solve_result *results, void *stream);

/* Allocation-free variant of fm_apply_operator, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, result and errors as
 * fm_apply_operator.  Its scratch (the energies on the device and the two
 * coupling slots, 2 * nbatch * N doubles) lives in one static device array of
 * 64 MiB (8 Mi doubles, the first 4096 for the energies) per GPU, held until
 * the process ends; nothing is allocated or freed.  FM_E_INVALID when
 * nbatch > 4096 or 2 * nbatch * N > 8 Mi - 4096.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (several threads or streams) race;
 * calls one after another are safe, each clearing the slots it uses.  Returns
 * after the stream has finished the work. */
fm_status fm_apply_operator_noalloc(fm_problem *p, int nbatch, const double *E, const double *x_dev,
                                    double *y_dev, void *stream);

/* ---- Complex energies --------------------------------------------------
 *
 * The same linear systems (H - E S) c = b with E complex and b, c complex:
 * the paper's method works in complex arithmetic throughout (Sec. 4), and the
 * scattering problem of Sec. 2.1 is posed at a given energy E.  H and S are
 * real, so with c = c_re + i c_im the system is A(Re E) c_re + Im E S c_im =
 * b_re, A(Re E) c_im - Im E S c_re = b_im; the preconditioner's factors are
 * the real, energy-independent ones, and only its divide by
 * lambda_x + lambda_y - E becomes complex.  Complex vectors are stored as two
 * real rows per request: [request][re, im][N] (2N doubles per request).  The
 * products run in FP64 only.  No boundary condition other than the bound-state
 * one of fm_create_problem is built. */

/* y = (H - E S) x for nbatch complex requests.  E_re, E_im: host arrays of
 * nbatch.  x_dev, y_dev: nbatch * 2N doubles, not overlapping.  Errors:
 * FM_E_INVALID, FM_E_HIP, FM_E_BUSY. */
fm_status fm_apply_operator_complex(fm_problem *p, int nbatch, const double *E_re, const double *E_im,
                                    const double *x_dev, double *y_dev, void *stream);

/* z = L(E)^-1 r for nbatch complex requests (either variant of
 * fm_apply_precond), FP64.  r_dev and z_dev may be the same buffer.  Errors as
 * fm_apply_operator_complex. */
fm_status fm_apply_precond_complex(fm_problem *p, int nbatch, const double *E_re, const double *E_im,
                                   const double *r_dev, double *z_dev, void *stream);

/* fm_solve for nbatch complex requests: right-preconditioned flexible GMRES on
 * the 2N real unknowns of each request (the real form of the complex system),
 * FP64 Arnoldi, true FP64 residual ||b - A x|| / ||b|| over both rows at every
 * restart.  opts->prec must be FM_FP64.  Results and errors as fm_solve;
 * min_abs_denominator is the least modulus of lambda - E over the divide. */
fm_status fm_solve_complex(fm_problem *p, int nbatch, const double *E_re, const double *E_im, const double *b_dev,
                           double *x_dev, const fm_solve_opts *opts, fm_solve_result *results, void *stream);

/* y = S x for nbatch requests: S holds the basis products at the collocation
 * points (Sec. 3.1; the right-hand matrix of H c = E S c), block diagonal over
 * (alpha, M').  x_dev, y_dev: nbatch * N doubles, not overlapping.  Errors:
 * FM_E_INVALID, FM_E_HIP, FM_E_BUSY. */
fm_status fm_apply_mass(fm_problem *p, int nbatch, const double *x_dev, double *y_dev, void *stream);

/* ---- Bound-state energies: shift-invert Arnoldi ------------------------
 *
 * The eigenvalues E of H c = E S c nearest a shift sigma (Sec. 3.1,
 * eq. (FM-lin); Sec. 4 iterates with the inverse of H - E* S by implicitly
 * restarted Arnoldi).  They are the eigenvalues theta = 1/(E - sigma) of
 * largest modulus of T = (H - sigma S)^-1 S.  Each Arnoldi step applies S and
 * solves with H - sigma S by fm_solve's flexible GMRES (opts->inner); the
 * basis stays on the device and is orthogonalised twice by classical
 * Gram-Schmidt.  Restarts are Krylov-Schur restarts (equivalent to the
 * implicit shifts of IRAM): the Ritz vectors of the nev + (ncv - nev)/2
 * largest |theta| (complex pairs kept whole) are orthonormalised and the basis
 * is contracted onto them.  A Ritz pair is accepted when the Arnoldi estimate
 * ||T V y - theta V y|| <= tol |theta| (||y|| = 1). */
typedef struct {
    int nev;                  /* eigenvalues wanted, nearest sigma */
    int ncv;                  /* Krylov basis size: nev + 2 <= ncv <= min(256, N) */
    double tol;               /* relative Ritz residual */
    int max_restarts;
    fm_solve_opts inner;      /* solves with H - sigma S (x0_is_guess ignored) */
} fm_eigs_opts;

typedef struct {
    int nconv;                /* wanted eigenvalues whose Ritz pairs met tol */
    int restarts;
    int solves;               /* Arnoldi steps (one inner solve each) */
    long long inner_iters;    /* GMRES steps over all inner solves */
    int inner_failures;       /* inner solves that stopped short of their rtol */
} fm_eigs_info;

/* E_re, E_im, resid: host arrays of nev entries, nearest sigma first (resid:
 * the Arnoldi estimate relative to |theta|; NaN where the Krylov space held
 * fewer values).  vec_dev (NULL: not formed): nev * N doubles, unit-norm
 * coefficient vectors; a complex pair fills two consecutive slots with the
 * real and imaginary parts of the first value's vector.  v0_dev (NULL: all
 * ones): the start vector, N doubles.  The device workspace ((2 ncv + 2) N
 * doubles plus the inner solve's) is allocated per call.  Returns FM_OK when
 * the nev values converged, FM_E_NOT_CONVERGED otherwise (the estimates are
 * returned); FM_E_INVALID, FM_E_NOMEM, FM_E_HIP, FM_E_BUSY, FM_E_NONFINITE. */
fm_status fm_eigs(fm_problem *p, double sigma, const fm_eigs_opts *opts, const double *v0_dev, double *E_re,
                  double *E_im, double *resid, double *vec_dev, fm_eigs_info *info, void *stream);

/* ---- Serving: continuous batching of solve requests --------------------
 *
 * A server owns a device-memory budget and a set of lanes.  A lane is one
 * (problem description, precision, restart length) with its own HIP stream,
 * host thread and Krylov workspace; its slots are the requests of that shape
 * waiting when the lane is made (at least 2, at most max_batch, fewer when
 * one slot is large).  Lanes run concurrently, so their kernels overlap on
 * the device.  An idle lane keeps its workspace until a new lane needs the
 * memory; then the longest idle lanes give it back, as many as needed.  Problems (the
 * energy-independent factors of fm_create_problem) are cached by description.
 * A submitted request is admitted when its lane has a free slot and the
 * budget covers the lane's workspace (and the problem, if it is new); it joins
 * the lane at the lane's next restart boundary (a lane ends its cycle early,
 * after at least 24 Arnoldi steps, when requests wait for its free slots).
 * Each request is the same flexible GMRES solve as fm_solve; restarts may
 * differ from a solve alone, so a result alone and in a mix agree to the
 * solve's accuracy, not bitwise.  A request whose true residual falls by less
 * than a factor 10 over a full cycle has stalled at its restart length (GMRES(m)
 * can stagnate for energies high in the continuum): it leaves its lane and is
 * queued again with twice the restart length (up to 1000, and while one slot
 * fits a quarter of the budget), from x = 0, with the Arnoldi steps it has
 * left (at least the new restart length); its result reports the steps of
 * every lane and the restart length it finished with.  A request whose
 * footprint exceeds the whole budget is finished with FM_E_REJECTED. */
typedef struct fm_server fm_server;

typedef struct {
    uint64_t tag;             /* the caller's tag from fm_submit */
    int status;               /* fm_status of the request */
    int iters;                /* Arnoldi steps (all lanes it ran in) */
    double rel_residual;      /* final true ||b - A x|| / ||b|| */
    double t_submit, t_start, t_done;  /* seconds (steady clock): submitted, joined a lane, finished */
    int restart;              /* restart length of the lane it finished in (the submitted one, or
                                 larger after stalls) */
} fm_request_result;

/* hbm_budget_bytes: device bytes the server may hold (factors + workspaces).
 * max_batch: most slots per lane (>= 1).  device: HIP device ordinal.
 * Errors: FM_E_INVALID, FM_E_HIP, FM_E_NOMEM. */
fm_status fm_server_create(size_t hbm_budget_bytes, int max_batch, int device, fm_server **out);

/* Queue one solve.  b_host (N doubles) is copied before the call returns;
 * x_host (N doubles) receives the solution and must stay valid until the
 * request's result has been returned by fm_poll.  Non-blocking.
 * Errors: FM_E_INVALID (bad arguments, server shutting down), FM_E_NOMEM. */
fm_status fm_submit(fm_server *s, const fm_problem_desc *desc, double E, const double *b_host, double *x_host,
                    const fm_solve_opts *opts, uint64_t tag);

/* Move up to max finished results into results[], *n_done of them.  With
 * block != 0, wait until at least one result is ready or nothing is
 * outstanding.  Errors: FM_E_INVALID. */
fm_status fm_poll(fm_server *s, fm_request_result *results, int max, int *n_done, int block);

/* Device bytes held, live lanes, requests submitted and not yet finished. */
fm_status fm_server_stats(fm_server *s, size_t *bytes_in_use, int *lanes, long long *outstanding);

/* Drain: every submitted request is finished, then all threads, lanes and
 * cached problems are released.  Results not yet polled are discarded. */
fm_status fm_server_destroy(fm_server *s);

/* Per-kernel-class timing of the calls above, for roofline accounting.
 * While enabled, HIP events are recorded on the caller's stream around every
 * kernel launch (a few microseconds per launch), and the algorithmic bytes
 * and flops of each launch are added up from the problem sizes and the number
 * of Arnoldi steps each request took (unique FP64 words read and written by
 * the operation's definition; caches and re-reads not counted).
 * fm_profile(p, 1) resets the counters and enables; fm_profile(p, 0) disables.
 * fm_profile_read returns, for one class, the summed kernel time in ms, the
 * number of launches, and the algorithmic bytes and flops. */
typedef enum {
    FM_K_MATVEC = 0,    /* operator (H - E S) x */
    FM_K_MODEZ = 1,     /* preconditioner z-mode products */
    FM_K_XY = 2,        /* preconditioner x-y slice products and divide */
    FM_K_MDOT = 3,      /* Arnoldi dot pass: basis^T [new direction, its image] */
    FM_K_MUPDATE = 4,   /* Arnoldi update pass: normalise the direction, project the image */
    FM_K_FINISH = 5,    /* per-request step completion: Hessenberg column, Givens, residual estimate */
    FM_K_RESTART = 6,   /* per-cycle solution update and true residual */
    FM_K_COUPLING = 7,  /* operator: coupling to the other components (FM_K_MATVEC: the rest) */
    FM_K_COUNT = 8
} fm_kernel_class;

fm_status fm_profile(fm_problem *p, int enable);
fm_status fm_profile_read(const fm_problem *p, int kclass, double *total_ms, long long *launches, double *bytes,
                          double *flops);

#ifdef __cplusplus
}
#endif

#endif /* FM_H */

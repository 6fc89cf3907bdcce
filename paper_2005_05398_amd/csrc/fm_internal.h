// Internal declarations of the FM solver library (host setup, device
// descriptors, kernel launchers).  Not part of the public ABI (include/fm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fm.h"

namespace fm {

constexpr int MAXR = 6;      // at most 2q = 6 nonzero 1D basis functions per point
constexpr int MAXM = 16;     // at most 16 M' blocks (J <= 15)

// ---------------------------------------------------------------------------
// Host: 1D Hermite spline basis with Gauss collocation points.
struct Basis1D {
    int degree = 0, q = 0, n = 0, K = 0;
    bool dirichlet = false;      // x, y: value function dropped at both ends
    double R = 0, lo = 0, hbar = 0;
    std::vector<double> nodes;   // K + 1
    std::vector<double> points;  // n collocation points, increasing
    std::vector<int> idx;        // n * MAXR global function index per local slot (-1: none)
    std::vector<double> val[3];  // n * MAXR values of the 0th, 1st, 2nd derivative

    int half = 0;                // z on [0, 1] with a parity at z = 0: +1 even, -1 odd (0: not halved)
    // Returns "" on success or a message.
    std::string init(const fm_dim &d, bool is_z);
    // The z basis on [0, 1] of a function of parity sigma about z = 0, on the
    // nodes and points of the full z basis d (an even number of intervals)
    // that lie in [0, 1]: at the node z = 0 the functions of odd derivative
    // order (sigma = +1) or of even order (sigma = -1) are dropped.
    std::string init_half(const fm_dim &d, int sigma);
    int global_index(int m, int d) const;
    int interval(double t) const;
    // Values of the 2q local functions (slot e*q + d) at t; gidx may be null.
    void eval_local(double t, int deriv, int *gidx, double *v) const;
    // Dense n x n matrix of the deriv-th derivative at the collocation points.
    std::vector<double> dense(int deriv) const;
};

// ---------------------------------------------------------------------------
// Host dense linear algebra (row-major n x n).
// All eigenvalues of the real matrix A ordered by decreasing modulus (a complex
// pair as a + ib, a - ib with b > 0), and unit eigenvectors of the leading ones
// by inverse iteration (up to ncols columns, pairs whole: a pair gives the real
// and imaginary parts of the first value's vector, type 1 and 2; a real value
// type 0) in the nv columns of V (row-major n x nv).  A vector whose residual
// exceeds 1e-11 max(|A|, |lambda|) ends the list; fewer than nmin columns is
// an error.  Returns "" or a message.
std::string dense_eig_by_modulus(int n, const std::vector<double> &A, int nmin, int ncols, std::vector<double> &wr,
                                 std::vector<double> &wi, std::vector<double> &V, std::vector<signed char> &type,
                                 int &nv);
bool lu_factor(int n, std::vector<double> &a, std::vector<int> &piv);
void lu_solve(int n, const std::vector<double> &lu, const std::vector<int> &piv, double *b);
bool invert(int n, const std::vector<double> &a, std::vector<double> &inv);

// Real quasi-diagonalisation of the pencil (A1, A2), A2 nonsingular:
//   Wbar A1 W = Lambda,  Wbar A2 W = I,
// Lambda block diagonal with 1x1 real blocks and 2x2 blocks [[a, b], [-b, a]]
// for complex pairs a +- ib.  type[i] = 0 (real), 1 (first of a pair),
// 2 (second); lre[i] = a (or the real eigenvalue), lim[i] = b for the first of a
// pair, -b for the second, 0 otherwise.  Eigenvalues ordered by increasing real
// part.  Returns "" or a message; err receives the check residual.
std::string pencil_diag(int n, const std::vector<double> &A1, const std::vector<double> &A2,
                        std::vector<double> &Wbar, std::vector<double> &W, std::vector<double> &lre,
                        std::vector<double> &lim, std::vector<signed char> &type, double *err);

// ---------------------------------------------------------------------------
// Device descriptors (plain data, passed by value to kernels).
struct DimDev {
    int n, K, q, drop0;          // drop0 = 1: the node-value function at both ends is absent
    double R, lo, hbar;
    const double *nodes;         // K + 1
    const double *pts;           // n
    const int *idx;              // n * MAXR
    const double *S, *D1, *D2;   // n * MAXR
    const int *first, *last;     // n: first and last global function index nonzero at each point
};

struct CompDev {
    DimDev x, y, z;
    long long off;               // offset of component alpha in one request vector
    int nxy, npts;               // nx*ny, nz*nx*ny (one M' block)
    const double *P;             // potential field V_a + sum_b V_b^(l), npts
    const double *Vs;            // V_a^(s)(x, y), nx*ny
    double c[3], s[3];           // (c_ba, s_ba) for beta = 0..2
    int xt;                      // x points per matvec tile
    int ntiles;                  // matvec tiles of this component: nz * ceil(nx / xt)
    // x groups: runs of consecutive points with the same x support (<= 4 points)
    const int *xg;               // ngx + 1 group starts (xg[ngx] = nx)
    int ngx, gt;                 // number of groups, groups per grouped tile
    int ntiles_g;                // grouped tiles: nz * ceil(ngx / gt)
};

// One grouped operator tile: component, z point, first x group and number of
// groups, the tile's x points [ixs, ixe) and their x support [kxlo, kxhi].
constexpr int GT_REC = 8;
enum { GT_A = 0, GT_IZ, GT_G0, GT_NGT, GT_IXS, GT_IXE, GT_KXLO, GT_KXHI };

// Coupling pairs grouped by (beta, cell of beta); built on the host.
// One coupling task (a (beta, cell) group of at most 64 pairs): everything a
// wave needs before it can fetch the cell's coefficients, so that the fetch
// waits for this record only.
constexpr int CPL_TASK = 32;     // ints per task record
enum {
    CT_BETA = 0, CT_MZ, CT_MX, CT_MY, CT_FIRST, CT_COUNT,
    CT_NX, CT_NY, CT_NPTS, CT_OFF_LO, CT_OFF_HI,
    CT_FIDX = 11,                // 2 q_z z, 2 q x, 2 q y global function indices (-1: dropped)
    CT_SPLIT = 30,               // job records: 1 when the job's two halves hold a task each
    CT_TASK = 31                 // the task's index (its cell widths in r), -1 in an empty record
};
static_assert(CT_FIDX + 3 * MAXR <= CT_SPLIT, "function indices overlap the job fields");

struct CouplingDev {
    int ntasks;
    int njobs;                   // wave jobs: one task, or (one M'' block) two, one per half-wave
    int pairs_per_lane;          // 2: every job two tasks of <= 64 pairs; 1: paired tasks have <= 32
    // one M'' block: [njobs][2][CPL_TASK], the records of each job's two halves,
    // so that a lane finds its task without a dependent read; a job of one task
    // repeats its record in the second half (CT_SPLIT 0, the task over the whole
    // wave) or, with two pairs per lane, has an empty one (count 0, CT_TASK -1).
    // More M'' blocks: null; job j is task j.
    const int *jrec;
    long long npairs;
    const int *task;             // [ntasks][CPL_TASK] records (layout above); more M'' blocks only (else null)
    const double *r;             // [ntasks][3] cell width / hbar in z, x, y
    const int *out;              // [npairs] 2 * (alpha output index of M' block 0) + slot
    const double *s;             // [3][npairs] position inside the cell: z, x, y
    const double *F;             // [nM * nM][npairs] factor of beta's M'' value in alpha's M' row
};

struct ProblemDev {
    CompDev comp[3];
    int nM, J, tau, M0;
    long long N;                 // unknowns per request
    // angular coupling constants (L > 0)
    double lhp[MAXM], lhm[MAXM]; // lambda-hat^{J, M'} and lambda-hat^{J, -M'} per M' index
    double dcoef[MAXM * MAXM * 2 * MAXM]; // Wigner-sum coefficient table (see setup): 2J + 1 <= 2 MAXM terms
    int dlen;
    int q[3];                    // spline order of x, y, z (same for all components), 0 if mixed
    const int *gtile;            // [sum ntiles_g][GT_REC] grouped tiles, in launch order (layout below)
    int tile_lds;                // doubles of LDS: the larger of the two below
    int plane_lds;               // doubles of LDS for the z-contracted planes of k_local_tiled
    int group_lds;               // doubles of LDS for the planes and x rows of k_local_grouped
    int lds_max;                 // bytes of LDS one block may use on the device
    int nodes_total;             // doubles of LDS for all node tables
    CouplingDev cpl;             // tiled path only
    const ProblemDev *dev;       // device copy of this descriptor (kernels take this pointer)
};

// The operator runs as two tiled kernels (coupling into a two-slot buffer, then
// the local stencil plus that buffer) when x and y share one spline order in
// all components, z one order, 2q <= n_y <= 256 and the operator's
// z-contracted planes fit the LDS of one block (n_M <= 3: kernels specialised
// for the block count; more blocks: kernels that take them one at a time);
// otherwise one generic kernel does everything.
inline bool matvec_tiled_ok(const ProblemDev &pd) {
    const bool same_xy = pd.q[0] != 0 && pd.q[0] == pd.q[1];
    bool rows_fit = true;                // one block of 256 threads covers the y points
    for (int a = 0; a < 3; ++a) rows_fit = rows_fit && pd.comp[a].y.n <= 256;
    return same_xy && rows_fit && pd.q[2] != 0 && pd.nM <= MAXM && sizeof(double) * size_t(pd.tile_lds) <= size_t(pd.lds_max);
}

struct PrecCompDev {
    int nx, ny, nz, nM;
    const double *Wz;            // [nM][2][nz][nz]  (0: Wbar_z, 1: W_z)
    const double *Wx;            // [nM][nz][2][nx][nx]
    const double *Wy;            // [nM][nz][2][ny][ny]
    const double *lx, *lxi;      // [nM][nz][nx]
    const double *ly, *lyi;      // [nM][nz][ny]
    const signed char *tx, *ty;  // [nM][nz][nx], [nM][nz][ny]
    const float *Wz32, *Wx32, *Wy32;          // FP32 copies
    const unsigned short *Wx16, *Wy16;        // BF16 planes [hi | mid], each laid out as Wx / Wy
    // coupled variant: joint z matrices [2][nM nz][nM nz] (0: forward, 1: backward);
    // the x-y factors above are then indexed by slot (l, m) instead of (M', k)
    const double *Zj;
};

struct PrecDev {
    PrecCompDev comp[3];
    int coupled;                 // 1: coupled variant (joint z matrices), 0: block-Jacobi in M'
    const int *pair_slices;      // slices (numbered over the components) whose x or y pencil has
    int npair_slices;            // complex eigenpairs; the staged divide leaves their blocks to k_divide_pairs
    const PrecDev *dev;          // device copy of this descriptor
};

// Per-call GMRES device state (pointers into one allocation).
struct KrylovDev {
    int nb, m;
    long long N;
    double *V;                   // [m+1][nb][N]
    double *Z;                   // [m][nb][N]
    double *H;                   // [nb][m+1][m]   (rotated: upper triangle R)
    double *g;                   // [nb][m+1]
    double *cs, *sn;             // [nb][m]
    double *hcol;                // [nb][m+1] t and c of the last step (its column before the delayed part)
    double *hproj;               // [nb][m+1] s of the last step (second projection of its direction)
    double *y;                   // [nb][m]
    double *part;                // [nb][2m+3][NBLK] reduction partials
    unsigned *ticket;            // [nb]
    int *active;                 // [nb] 1 while the request iterates in this cycle
    int *jcount;                 // [nb] Arnoldi steps in this cycle
    double *bnorm, *rnorm;       // [nb]
    double *scal;                // [nb] r_j of the last step
    double *rho;                 // [nb] scale of the newest direction
    double *E;                   // [nb]
    double *tol;                 // [nb] absolute inner tolerance
    int *flags;                  // [nb] breakdown / nonfinite flags
    int *closed;                 // [nb] 1: the cycle ended on its closing pass (not on convergence)
};

constexpr int NBLK = 1024;       // at most this many blocks per request in the reduction kernels
constexpr int MAX_RESTART = 1000;

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip).
// part: 0 whole operator, 1 everything but the coupling, 2 the coupling.  On the
// tiled path part 2 writes the coupling of every request into cbuf
// ([nb][2][N], slot = which partner) and part 1 adds cbuf to the local operator,
// so part 2 must run first; entries of cbuf that no coupling pair writes must be
// zero (they stay so).  The generic path ignores cbuf and does it all in part 1.
void launch_matvec(const ProblemDev &pd, int nb, const double *E_dev, const int *active,
                   const double *x, double *y, double *cbuf, hipStream_t st, int part = 0);
void launch_zjoint(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which, const double *in,
                   double *out, hipStream_t st);
void launch_modez(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which,
                  const double *in, double *out, hipStream_t st);
// tmp ([nb][N] scratch): the four products run as batched GEMMs through tmp
// over all slices at once when a slice side exceeds XY_FUSED_MAX_SIDE;
// otherwise one block per slice does all four in LDS, however few the slices
// (measured faster from 24 slices up: a single launch instead of five).
constexpr int XY_FUSED_MAX_SIDE = 32;
// BF16x3 products: the staged chain below this many slices (measured faster at
// 384 slices of side 31; FP64 and FP32 take the fused kernel at any count)
constexpr long long XY_BF16_FUSED_FROM = 512;
constexpr long long XY_T64_MIN_BLOCKS = 1024;  // staged products: 64 x 64 tiles from this many blocks
void launch_xy(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active,
               double *data, double *min_den, double *tmp, hipStream_t st);
// reduced-precision products (mode 1: FP32 MFMA, 2: BF16x3 MFMA); false if the slice does not fit
void launch_modez_lp(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which,
                     const double *in, double *out, hipStream_t st);
bool launch_xy_lp(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active,
                  double *data, int mode, double *tmp, hipStream_t st);
// The reduced-precision preconditioner (mode 1: FP32 MFMA, 2: BF16x3 MFMA)
// with FP32 storage between its products, in three launches: the z product
// (which 0: in -> the FP32 view of tmp; the coupled variant's joint z product
// stays FP64, in -> tmp), the four staged x-y products through the FP32 views
// of out and tmp with the FP64 divide, and the z product back (which 1: into
// out, FP64).  in may equal out; tmp: [nb][N] doubles.  precond_f32_ok: the
// staged products (for this mode) and the register z product apply (else the
// caller runs the FP64-storage path).
bool precond_f32_ok(const ProblemDev &pd, const PrecDev &pr, int nb, int mode);
void launch_z_f32(const ProblemDev &pd, const PrecDev &pr, int nb, const int *active, int which, const double *in,
                  double *out, double *tmp, hipStream_t st);
void launch_xy_f32(const ProblemDev &pd, const PrecDev &pr, int nb, const double *E_dev, const int *active, int mode,
                   double *out, double *tmp, hipStream_t st);
// Arnoldi / GMRES pieces (V and Z stored [i][request][N])
// Step j: dot pass over slots 0..j+1 (0..j when closing), then the per-request
// finish (Hessenberg column j - 1, Givens, stop test), then the update pass.
void launch_arnoldi_dots(const KrylovDev &k, int j, int closing, hipStream_t st);
void launch_arnoldi_finish(const KrylovDev &k, int j, int closing, hipStream_t st);
void launch_arnoldi_update(const KrylovDev &k, int j, hipStream_t st);
void launch_cycle_solve(const KrylovDev &k, const int *running, hipStream_t st);
void launch_xupdate(const KrylovDev &k, const int *running, double *x, hipStream_t st);
void launch_residual(const KrylovDev &k, int *running, const double *b, double rtol, double inner_safety,
                     hipStream_t st);
void launch_scale0(const KrylovDev &k, hipStream_t st);
// y = S x (the mass matrix of H c = E S c) for nb requests; active (may be
// null): the requests to compute (the others' rows of y are left as they are)
void launch_mass(const ProblemDev &pd, int nb, const double *x, double *y, hipStream_t st,
                 const int *active = nullptr);
// Column kernels of the eigenvalue iteration (columns of length N stored one after another):
// out[c] = V_c . w (part: cols_dot_blocks(N) * ncol doubles of scratch); w -= V h (h on the
// device); out_c = sum_j V_j Y[j k + c] (Y on the device, row-major m x k; out must not
// overlap V); w *= s.
int cols_dot_blocks(long long N);
void launch_cols_dot(const double *V, int ncol, const double *w, long long N, double *part, double *out,
                     hipStream_t st);
void launch_cols_axpy(double *w, const double *V, int ncol, const double *h, long long N, hipStream_t st);
void launch_cols_combine(const double *V, int m, const double *Y, int k, double *out, long long N, hipStream_t st);
void launch_scale_vec(double *w, double s, long long N, hipStream_t st);
void launch_bnorm(const KrylovDev &k, const double *b, const int *mask, hipStream_t st);
void launch_zero_start(const KrylovDev &k, double *x, const int *mask, int zero_x, hipStream_t st);
void launch_fill(double *p, long long n, double v, hipStream_t st);
void prepare_large_lds(size_t bytes);
// Allows the tiled operator kernels dynamic LDS above 64 KB.
void prepare_operator_lds(size_t bytes);
size_t xy_lds_limit();
void launch_copy(double *dst, const double *src, long long n, hipStream_t st);
// Complex energies: a complex request is two rows (real, imaginary part).
// The divide of the preconditioner with E complex, in place over the slices
// of nbc complex requests (active: per complex request; min_den: [nbc]).
void launch_cdivide(const ProblemDev &pd, const PrecDev &pr, int nbc, const double *Ere, const double *Eim,
                    const int *active, double *data, double *min_den, hipStream_t st);
// y_re += E_im sx_im, y_im -= E_im sx_re (sx = S x of both rows).
void launch_cplx_energy(double *y, const double *sx, const double *Eim, const int *active, int nbc, long long N,
                        hipStream_t st);
// out[2c] = out[2c + 1] = in[c] for c < n.
void launch_expand_mask(const int *in, int *out, int n, hipStream_t st);
// The forward (which 0) or backward (which 1) pair of staged x-y products over
// nrows rows, data -> tmp -> data, with no divide.
void launch_xy_half(const ProblemDev &pd, const PrecDev &pr, int nrows, const int *active, int which, double *data,
                    double *tmp, hipStream_t st);

}  // namespace fm

/*
 * fm_host.h - host-only inspection of the set-up stages of libfm (no device
 * is touched).  These run the same code that fm_create_problem uses, so the
 * 1D bases and the pencil diagonalisation can be checked on a machine
 * without a GPU.
 */
#ifndef FM_HOST_H
#define FM_HOST_H

#include "fm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The collocation points and the n x n matrices S, D1, D2 (row = point,
 * column = basis function, row-major) of one 1D basis (Sec. 3.1: (S)_{pk} =
 * S^k(t_p), (D)_{pk} = S^k''(t_p); Sec. 3.3: D_1 the first derivative).
 * is_z selects the z closure.  Output arrays hold n and n*n doubles; any may
 * be NULL.  Errors: FM_E_INVALID for an inadmissible basis. */
fm_status fm_host_basis(const fm_dim *dim, int is_z, double *points, double *S, double *D1, double *D2);

/* D(A1, A2) of Sec. 3.2, eq. (WW-scale), in real arithmetic: Wbar A1 W =
 * Lambda, Wbar A2 W = I with Lambda quasi-diagonal (2x2 blocks [[a, b],
 * [-b, a]] for complex pairs a +- ib).  A1, A2, Wbar, W: n*n row-major; lre,
 * lim: n doubles (lim = b, -b on the two rows of a pair, 0 otherwise); type:
 * n bytes (0 real, 1 first of a pair, 2 second).  err receives the relative
 * residual of the two identities.  Errors: FM_E_PENCIL. */
fm_status fm_host_pencil(int n, const double *A1, const double *A2, double *Wbar, double *W, double *lre,
                         double *lim, signed char *type, double *err);

/* Build every pencil factor of a problem on the host and report the largest
 * relative residual of the diagonalisations, the number of complex pairs
 * among the x and y pencils, and N.  Errors as fm_create_problem, without
 * FM_E_HIP / FM_E_NOMEM. */
fm_status fm_host_setup_check(const fm_problem_desc *desc, double *max_err, int *complex_pairs, size_t *n_unknowns);

/* The coupling term of the operator (the off-diagonal blocks in alpha of
 * H - E S: V_alpha^(s) times the partners' expansions at the rotated points,
 * Sec. 2 and eq. (FM-pre)) applied to x, evaluated on the host from the same
 * grouped coupling pairs that the device operator uses, walked as the device
 * kernels walk them (per wave job and lane, from the task record that lane
 * reads): y = C x (N doubles each; both may be NULL to count only).  npairs:
 * (point, partner) pairs with a nonzero factor inside the partner's box;
 * ntasks: groups of at most 64 pairs that share one partner cell.  Errors as
 * fm_host_setup_check, and FM_E_INVALID if the jobs do not take every pair
 * exactly once. */
fm_status fm_host_coupling(const fm_problem_desc *desc, const double *x, double *y, long long *npairs, int *ntasks);

/* z = L(E)^-1 r for one request on the host, from the same factor tables that
 * fm_create_problem uploads and in the order the device applies them: the z
 * transform (per M' block, or the coupled variant's joint matrix), then per
 * x-y slice Wbar_x T Wbar_y^T, the divide by lambda_x + lambda_y - E and
 * W_x T W_y^T, then the z transform back (fm_apply_precond describes both
 * variants).  r, z: N doubles each, not overlapping.  For checking the set-up
 * only: plain loops, small problems.  Errors as fm_host_setup_check, and
 * FM_E_PENCIL when an x or y pencil has complex pairs (not handled here). */
fm_status fm_host_precond(const fm_problem_desc *desc, double E, const double *r, double *z);

/* The eigenvalues of the x and y pencils of one x-y slice, as the divide of
 * fm_apply_precond uses them (Sec. 3.2, eq. (prec-2)): the denominator of the
 * slice's element (i, j) is lx_re[i] + ly_re[j] - E for real eigenvalues
 * (lx_im, ly_im zero; a complex pair holds +b, -b on its two rows).  alpha:
 * component 0..2; slot: 0 .. n_M n_z - 1 (M' n_z + k for the block-Jacobi
 * variant, the coupled variant's (l, m) slots in the same numbering).  Output
 * arrays hold n_x and n_y doubles; any may be NULL.  Errors as
 * fm_host_setup_check, FM_E_INVALID for alpha or slot out of range (or a
 * component implied by the exchange symmetry). */
fm_status fm_host_slice_eigenvalues(const fm_problem_desc *desc, int alpha, int slot, double *lx_re, double *lx_im,
                                    double *ly_re, double *ly_im);

#ifdef __cplusplus
}
#endif

#endif /* FM_HOST_H */

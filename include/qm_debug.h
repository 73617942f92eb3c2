/*
 * qm_debug.h -- host-only diagnostic entry points of libqm (no device work).
 * They expose the table builders' intermediate results (Student t, and the
 * exponential -> hyperbolic map) so that their accuracy can be checked on a
 * machine without a GPU.
 */
#ifndef QM_DEBUG_H
#define QM_DEBUG_H

#ifdef __cplusplus
extern "C" {
#endif

/*
 * The builder's dense solution of the Gaussian-background recycling ODE for
 * the Student t target (Section 3.1), q[i] = Q(z[i]) for |z[i]| <= 40,
 * from the same forward/backward Taylor-series integration that feeds the
 * table (in __float128, rounded; the backward leg starts just past the
 * largest |z[i]|, at 10.5 at least).  nu in [0.5, 1e5].  Host arrays of n
 * doubles.  Returns 0, or -1 for an unsupported nu or |z[i]| > 40.
 */
int qm_debug_student_dense(double nu, const double* z, double* q, int n);

/*
 * Build the table for nu on the host.  header_out (may be NULL) receives the
 * table header (struct qm::TTableHeader of csrc/qm_table.h, 200 bytes: the
 * tail constants and, for FP64 and FP32 outputs, the cell layout with the
 * builder's self-checked fit error); coef_out (may be NULL) receives the
 * coefficient block (both cell sets, at their coef_offset) if coef_cap
 * doubles are enough.  Returns the number of doubles in the block, or -1 if
 * the build failed.
 */
int qm_debug_student_table(double nu, void* header_out, double* coef_out, int coef_cap);

/*
 * The hyperbolic builder's solution of the exponential-background recycling
 * ODE (Section 8.1), q[i] = Q(v[i]) for |v[i]| <= 1e12: the Taylor-series
 * legs of each side within its anchor, the direct solution of the tail
 * condition beyond (in __float128, rounded).  Parameters as for
 * qm_hyperbolic_table_build.  Host arrays of n doubles.  Returns 0, or -1
 * for invalid parameters, |v[i]| > 1e12 or a failed solve (reason on
 * stderr).
 */
int qm_debug_hyperbolic_dense(double alpha, double beta, double delta, const double* v, double* q, int n);

/*
 * Build the hyperbolic table on the host.  header_out (may be NULL)
 * receives the header (struct qm::HypTableHeader of csrc/qm_hyp_table.h,
 * 392 bytes: parameters, the two sides' masses, and for each side and each
 * cell set -- FP64 outputs, FP32 outputs -- the cell layout, large-v
 * constants and the builder's check of its rounded rows); coef_out (may be
 * NULL) receives the rows of all four, at their coef_offset, if coef_cap
 * doubles are enough.  Returns the number of
 * doubles, or -1 if the build failed.
 */
int qm_debug_hyperbolic_table(double alpha, double beta, double delta, void* header_out, double* coef_out,
                              int coef_cap);

/* The same for the variance-gamma table of (lambda, alpha, beta), real
   lambda in [1, 8] (the header's delta field holds lambda). */
int qm_debug_vg_table(double lambda, double alpha, double beta, void* header_out, double* coef_out, int coef_cap);

#ifdef __cplusplus
}
#endif

#endif /* QM_DEBUG_H */

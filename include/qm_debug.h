/*
 * qm_debug.h -- host-only diagnostic entry points of libqm (no device work).
 * They expose the Student t table builder's intermediate results so that its
 * accuracy can be checked on a machine without a GPU.
 */
#ifndef QM_DEBUG_H
#define QM_DEBUG_H

#ifdef __cplusplus
extern "C" {
#endif

/*
 * The builder's dense solution of the Gaussian-background recycling ODE for
 * the Student t target (Section 3.1), q[i] = Q(z[i]) for |z[i]| <= 10.5,
 * from the same forward/backward Taylor-series integration that feeds the
 * table (in __float128, rounded).  nu in [0.5, 1e5].  Host arrays of n
 * doubles.  Returns 0, or -1 for an unsupported nu.
 */
int qm_debug_student_dense(double nu, const double* z, double* q, int n);

/*
 * Build the table for nu on the host.  header_out (may be NULL) receives the
 * table header (struct qm::TTableHeader of csrc/qm_table.h, 104 bytes); coef_out (may be NULL)
 * receives ncell * stride coefficients if coef_cap is large enough;
 * max_rel_err (may be NULL) the builder's self-checked fit error.  Returns
 * the number of coefficients, or -1 if the build failed.
 */
int qm_debug_student_table(double nu, void* header_out, double* coef_out, int coef_cap,
                           double* max_rel_err);

#ifdef __cplusplus
}
#endif

#endif /* QM_DEBUG_H */

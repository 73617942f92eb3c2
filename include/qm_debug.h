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

#ifdef __cplusplus
}
#endif

#endif /* QM_DEBUG_H */

/*
 * qm_table.h -- layout of the normal -> Student t tables and their host
 * builder (no HIP dependency: the builder is plain C++ with __float128).
 */
#pragma once
#include <stdint.h>

namespace qm {

/*
 * Device-side table of the normal -> Student t map for one nu.
 *
 * For |z| <= s_max the map is t = z R(y), y = z^2, with R evaluated per
 * cell: y in [j h, (j+1) h), j < ncell, R = sum_k c_{j,k} d^k with
 * d = y - (j + 1/2) h.  Coefficients are stored cell-major, highest power
 * first, with a row stride of `stride` doubles (>= degree + 1).
 * Beyond s_max the far-tail form t = sqrt(nu) w^{-1/nu} (1 + ...) is used,
 * w = K q(|z|) (Section 3.3, 3.5), with K and the series coefficients below.
 */
struct TTableHeader {
    double nu;
    double h;           /* cell width in y = z^2 */
    double inv_h;
    double y_max;       /* = ncell * h */
    double log_K;       /* log of n sqrt(pi) Gamma(n/2)/Gamma((n+1)/2) */
    double tail_a[4];   /* far-tail series t = sqrt(nu) w^{-1/nu} (1 + sum a_k w^{2k/nu}) */
    int32_t ncell;
    int32_t degree;
    int32_t stride;
    int32_t identity;   /* nu = +inf: t = z */
};

/* Host-built table: header + ncell*stride coefficients (doubles). */
struct HostTTable {
    TTableHeader hdr;
    double* coef;       /* host copy, malloc'd */
    double max_rel_err; /* builder's self-check against its own dense output */
};

/* Build the table for nu on the host (qm_table.cpp). Returns 0 on success. */
int build_student_table(double nu, HostTTable* out, char* err, int errlen);
void free_student_table(HostTTable* t);

}  // namespace qm

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
 * For y = z^2 <= y_max the map is t = z R(y), with R evaluated per cell:
 * j = floor(y / h) (clamped to ncell - 1), R = sum_k c_{j,k} d^k with
 * d = y - (j h + centre_offset).  Coefficients are stored cell-major,
 * highest power first, with a row stride of `stride` doubles (>= degree + 1);
 * an FP32 copy of the same array follows at byte offset coef_f32_offset.
 * Beyond y_max the two-term tail t = sqrt(nu) w^{-1/nu} (1 + a w^{2/nu}),
 * w = K q(|z|) (Sections 3.3, 3.5), is used with log K and a = tail_a[0].
 */
struct TTableHeader {
    double nu;
    double h;           /* cell width in y = z^2 */
    double inv_h;
    double y_max;       /* = ncell * h */
    double centre_offset; /* cell centre = j h + centre_offset */
    double log_K;       /* log of n sqrt(pi) Gamma(n/2)/Gamma((n+1)/2) */
    double tail_a[4];   /* far-tail series t = sqrt(nu) w^{-1/nu} (1 + sum a_k w^{2k/nu}) */
    int32_t ncell;
    int32_t degree;
    int32_t stride;
    int32_t identity;   /* nu = +inf: t = z */
    uint64_t coef_f32_offset; /* bytes from the table start to the FP32 copy */
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

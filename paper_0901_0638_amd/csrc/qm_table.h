/*
 * qm_table.h -- layout of the normal -> Student t tables and their host
 * builder (no HIP dependency: the builder is plain C++ with __float128).
 */
#pragma once
#include <stdint.h>

namespace qm {

/* Polynomial degrees per cell.  FP64 outputs need R to about an ulp of
   FP64: degree 7 on narrower cells where at most T_LDS_CELLS_LOW of them
   cover y <= 100 (nu >= 3 or so), else degree 15 on wider ones.  FP32
   outputs are rounded once from an FP64 evaluation, so R to 1e-10 relative
   (far below the 6e-8 half-ulp of FP32) is enough: degree 7.  Degree 7
   halves the table reads and the Horner chain per element. */
constexpr int T_DEGREE_LOW = 7;
constexpr int T_DEGREE_HIGH = 15;
constexpr int T_DEGREE_F32 = T_DEGREE_LOW;
constexpr int T_LDS_CELLS_LOW = 200;

/* Smallest nu tabulated.  log R grows like y / (2 nu), so the cells in y
   that meet the tolerances multiply as nu falls: at nu = 0.3 the FP64 set
   needs 400 rows of degree 15 and the FP32 set 400 of degree 7 up to
   y = 100, 54 KB and 29 KB of LDS; from about nu = 0.27 down the FP32 set
   no longer fits its 720 rows (and the FP64 set its 480 soon after). */
constexpr double T_NU_MIN = 0.3;

/*
 * One piecewise-polynomial approximation of R(y) = t(z)/z, y = z^2 <= y_max:
 * cell j = floor(y / h) (clamped to ncell - 1) holds R = sum_k c_{j,k} d^k,
 * d = y - (j h + centre_offset).  Rows are cell-major, highest power first,
 * `stride` = degree + 1 doubles each, starting `coef_offset` doubles into
 * the table's coefficient block.  The first nlds cells (y <= y_lds, about
 * 100: every sample of a normal below 10 in magnitude) are the ones staged
 * in LDS; the rest extend the table to where the two-term tail formula
 * meets the same accuracy (at most y = 1600), read from global memory on
 * the rare path.
 */
struct TCells {
    double h;             /* cell width in y (a power of 2, so j h is exact) */
    double inv_h;
    double y_max;         /* = ncell * h; beyond it the far-tail formula */
    double y_lds;         /* = nlds * h */
    double centre_offset; /* cell centre = j h + centre_offset */
    double max_rel_err;   /* builder's check of the rounded coefficients */
    int32_t ncell;
    int32_t nlds;
    int32_t degree;
    int32_t stride;
    uint64_t coef_offset;
};

/*
 * Device-side table of the normal -> Student t map for one nu: two cell
 * approximations of the same map (FP64 outputs, FP32 outputs), and the
 * two-term tail t = sqrt(nu) w^{-1/nu} (1 + a w^{2/nu}), w = K q(|z|)
 * (Sections 3.3, 3.5), with log K and a = tail_a[0], used beyond y_max.
 * On the device the header is followed by the coefficient block.
 */
struct TTableHeader {
    double nu;
    double log_K;       /* log of nu sqrt(pi) Gamma(nu/2)/Gamma((nu+1)/2) */
    double tail_a[4];   /* far-tail series t = sqrt(nu) w^{-1/nu} (1 + sum a_k w^{2k/nu}) */
    int32_t identity;   /* nu = +inf: t = z */
    int32_t reserved;
    TCells f64;         /* degree T_DEGREE_LOW or T_DEGREE_HIGH */
    TCells f32;         /* degree T_DEGREE_F32 */
};

/* Host-built table: header + coefficient block (doubles). */
struct HostTTable {
    TTableHeader hdr;
    double* coef;       /* host copy, malloc'd */
    uint64_t ncoef;     /* doubles in the block (both approximations) */
};

/* Build the table for nu on the host (qm_table.cpp). Returns 0 on success. */
int build_student_table(double nu, HostTTable* out, char* err, int errlen);
void free_student_table(HostTTable* t);

}  // namespace qm

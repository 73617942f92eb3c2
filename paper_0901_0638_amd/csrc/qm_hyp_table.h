/*
 * qm_hyp_table.h -- layout of the exponential -> hyperbolic tables and their
 * host builder (plain C++ with __float128, no HIP dependency).
 */
#pragma once
#include <stdint.h>

namespace qm {

constexpr int HYP_DEGREE = 11;      /* polynomial degree per cell, FP64 outputs */
constexpr int HYP_DEGREE_F32 = 7;   /* FP32 outputs (cells to 1e-10, evaluated in FP64) */
constexpr int HYP_SUB = 8;          /* cells per octave (a power of 2) */
constexpr int HYP_MAX_OCT = 40;     /* octaves per side at most */

/*
 * One side of the map (v >= 0 with beta, or the mirrored v < 0 side with
 * -beta): Q(v) = v R(v) for 0 <= v < v_top, R in cells of the variable
 * t = 1 + v / v0 (v0 a power of 2, the same for both sides): HYP_SUB equal
 * cells in each octave [2^k, 2^(k+1)) of t, k < noct, so cell
 * j = HYP_SUB k + i is read off the exponent and leading mantissa bits of t.
 * Cell j holds R = sum_k c_{j,k} d^k, d = v - centre_j, centre_j at
 * t = 2^k (1 + (i + 1/2)/HYP_SUB), highest power first, degree + 1
 * doubles per row, starting coef_offset doubles into the table's
 * coefficient block.  A side with origin = 1 (a variance-gamma target
 * whose density carries |x|^rho at 0, rho = 2 lambda - 1 not an integer)
 * instead holds in row 0 the first octave v < v0 as one series in v and
 * w = v^rho, R = P0(v) + w (P1(v) + w (P2(v) + w P3(v))): rho, then the
 * coefficients of P3, P2, P1, P0, highest power first, degrees 4, 2, 1, 0
 * (FP64-output cells) or, without P3, 3, 1, 0 (FP32-output cells); rows 1
 * to HYP_SUB - 1 are then not read.  From v_top = v0 (2^noct - 1) on, the large-v
 * expansion of the tail condition: for the hyperbolic target (Section 8.1:
 * both H and the base have constant rates far out, so Q - v tends to a
 * constant) Q = v + far_c0 + (far_c1 + far_c2 / v) / v; for a target whose
 * tail carries a power of x, as variance-gamma's x^(lambda-1) (Section 8.2),
 * Q = v + far_c0 + far_clog log Q + (far_c1 + far_c2 / Q) / Q, by three
 * fixed-point steps from v + far_c0 + far_clog log v.
 */
struct HypSide {
    double v0, inv_v0, v_top;
    double far_c0, far_c1, far_c2;
    double far_clog;         /* 0: Q = v + c0 + (c1 + c2/v)/v; else the log form (qm_hyp_device.hpp) */
    double max_rel_err;      /* builder's check of the rounded coefficients */
    int32_t noct;
    int32_t ncell;           /* HYP_SUB noct */
    int32_t degree;          /* rows of degree + 1 doubles */
    int32_t origin;          /* 1: the first octave (v < v0) is the series in v and v^rho of row 0 */
    uint64_t coef_offset;
};

struct HypTableHeader {
    double alpha, beta, delta;        /* delta: lambda for a variance-gamma table */
    double log_p_plus, log_p_minus;   /* target masses on x > 0 and x < 0 */
    HypSide right;                    /* v >= 0, FP64 outputs (degree HYP_DEGREE, to 2e-17) */
    HypSide left;                     /* v < 0, as -Q(-v) of the mirrored side */
    HypSide right32, left32;          /* FP32 outputs (degree HYP_DEGREE_F32, to 1e-10) */
};

static_assert(sizeof(HypTableHeader) == 392, "the header layout is part of qm_debug.h");

struct HostHypTable {
    HypTableHeader hdr;
    double* coef;            /* malloc'd block of both sides' rows */
    uint64_t ncoef;
};

/* Build the table for (alpha, beta, delta), |beta| < alpha, delta > 0
   (qm_hyp_table.cpp).  Returns 0 on success. */
int build_hyperbolic_table(double alpha, double beta, double delta, HostHypTable* out, char* err, int errlen);
void free_hyperbolic_table(HostHypTable* t);

/* The same table format for the variance-gamma target (Section 8.2) with
   real lambda in [1, 8] and |beta| < alpha; the header's delta field
   holds lambda.  Returns 0 on success. */
int build_vg_table(double lambda, double alpha, double beta, HostHypTable* out, char* err, int errlen);

}  // namespace qm

/*
 * qm_student_device.hpp -- per-element evaluation of the normal -> Student t
 * map from a table staged in LDS (shared by the single-request and the
 * batch kernels).
 */
#pragma once
#include <hip/hip_runtime.h>

#include "qm_device.hpp"

namespace qm {

constexpr int T_DEGREE = 15;
constexpr int T_STRIDE = 16;

/* Uniform per-launch parameters (copied from the host-side header). */
struct StudentParams {
    double h, inv_h, centre_offset, y_max, log_K, tail_a, sqrt_nu, inv_nu, nu;
    int ncell;
    int identity;
    int lds_stride;   /* doubles between cell rows in LDS (>= T_STRIDE; padding spreads banks) */
};

/* Copy a table (ncell rows of T_STRIDE doubles) into LDS rows of P.lds_stride. */
__device__ __forceinline__ void stage_table(double* lds, const double* __restrict__ coef, const StudentParams& P)
{
    const int ncoef = P.ncell * T_STRIDE;
    for (int i = threadIdx.x; i < ncoef; i += blockDim.x) lds[(i >> 4) * P.lds_stride + (i & 15)] = coef[i];
}

/* Far tail (y > y_max): w = K q(s), q(s) = erfcx(s/sqrt2) e^{-s^2/2} / 2,
   t = sqrt(nu) w^{-1/nu} (1 + a w^{2/nu}) (Sections 3.3, 3.5).  log w is
   carried as a double-double (s^2/2 exactly, the division by nu with its
   remainder), because an absolute error e in it is a relative error e/nu
   in t and |log w| reaches several hundred. */
static __device__ __noinline__ double student_far(double s, const StudentParams& P)
{
#pragma clang fp contract(off)
    const double INV_SQRT2 = 0.70710678118654752440, LN2 = 0.69314718055994530942;
    if (!(s < __builtin_inf())) return s;              /* z = +-inf -> +-inf; NaN -> NaN */
    double hs = -0.5 * s;                              /* exact */
    double e_hi = hs * s;
    double e_lo = __builtin_fma(hs, s, -e_hi);         /* -s^2/2 = e_hi + e_lo exactly */
    double r = P.log_K + (::log(::erfcx(s * INV_SQRT2)) - LN2);
    double a_hi = e_hi + r;                            /* two-sum */
    double bb = a_hi - e_hi;
    double a_lo = (e_hi - (a_hi - bb)) + (r - bb) + e_lo;
    const double nu = P.nu;
    double q_hi = a_hi / nu;                           /* log w / nu = q_hi + q_lo */
    double q_lo = (__builtin_fma(-q_hi, nu, a_hi) + a_lo) / nu;
    double t = P.sqrt_nu * ::exp(-q_hi) * (1.0 - q_lo);
    return t * (1.0 + P.tail_a * ::exp(2.0 * q_hi));
}

/* t(z) in FP64 from the LDS table. */
__device__ __forceinline__ double student_eval(double z, const double* __restrict__ tab, const StudentParams& P)
{
    double s = __builtin_fabs(z);
    double yh = s * s;                      /* only selects the cell */
    double jd = yh * P.inv_h;
    const double jmax = (double)(P.ncell - 1);
    jd = (jd < jmax) ? jd : jmax;           /* NaN and inf clamp to the last cell */
    int j = (int)jd;
    double yc = __builtin_fma((double)j, P.h, P.centre_offset);   /* exact: h is a power of 2 */
    /* d = s^2 - y_c with a single rounding (|d| <= h/2): the full input
       precision reaches the polynomial, which matters because log R grows
       like y/(2 nu) */
    double d = __builtin_fma(s, s, -yc);
    const double* c = tab + j * P.lds_stride;
    double R = c[0];
#pragma unroll
    for (int k = 1; k <= T_DEGREE; ++k) R = __builtin_fma(R, d, c[k]);
    double t = z * R;
    bool far = !(yh <= P.y_max);            /* also NaN: NaN propagates either way */
    if (wave_any(far)) {
        double tf = __builtin_copysign(student_far(far ? s : 1.0, P), z);
        t = far ? tf : t;
    }
    return t;
}

}  // namespace qm

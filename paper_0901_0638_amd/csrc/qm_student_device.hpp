/*
 * qm_student_device.hpp -- per-element evaluation of the normal -> Student t
 * map from a table staged in LDS (shared by the single-request and the
 * batch kernels).
 */
#pragma once
#include <hip/hip_runtime.h>

#include "qm_device.hpp"

namespace qm {

/* Uniform per-launch parameters: the tail constants of the table header and
   the layout of the cell approximation in use. */
struct StudentParams {
    double h, inv_h, centre_offset, y_lds, y_max, log_K, tail_a, sqrt_nu, inv_nu, nu;
    const double* gcoef;  /* all ncell rows in global memory (the rare path reads them) */
    int ncell;        /* rows covering y <= y_max */
    int nlds;         /* rows staged in LDS, covering y <= y_lds */
    int identity;
    int row_shift;    /* log2 of the coefficients per row in memory (degree + 1) */
    int lds_stride;   /* doubles between cell rows in LDS: even, >= the row */
};

/* Copy the first nlds cell rows (2^row_shift doubles each) into LDS rows of
   P.lds_stride doubles. */
__device__ __forceinline__ void stage_table(double* lds, const double* __restrict__ coef, const StudentParams& P)
{
    const int ncoef = P.nlds << P.row_shift;
    const int mask = (1 << P.row_shift) - 1;
    for (int i = threadIdx.x; i < ncoef; i += blockDim.x) lds[(i >> P.row_shift) * P.lds_stride + (i & mask)] = coef[i];
}

/* R(y) of cell j by Horner in d = y - y_c (rows of DEG + 1 doubles). */
template <int DEG>
__device__ __forceinline__ double cell_poly(const double* __restrict__ c, double d)
{
    double R = c[0];
#pragma unroll
    for (int k = 1; k <= DEG; ++k) R = __builtin_fma(R, d, c[k]);
    return R;
}

/* The same from a row in LDS, read in 16-byte pieces (ds_read_b128): the
   rows start on 16-byte boundaries (even stride, 16-byte aligned LDS), so
   lanes on different cells either share a 16-byte bank group or none. */
template <int DEG>
__device__ __forceinline__ double cell_poly_lds(const double* __restrict__ row, double d)
{
    static_assert((DEG + 1) % 2 == 0, "rows of an even number of doubles");
    typedef double d2v __attribute__((ext_vector_type(2)));
    double c[DEG + 1];
#pragma unroll
    for (int k = 0; k < (DEG + 1) / 2; ++k) {
        const d2v x = *reinterpret_cast<const d2v*>(row + 2 * k);
        c[2 * k] = x.x;
        c[2 * k + 1] = x.y;
    }
    return cell_poly<DEG>(c, d);
}

/* Cell index and offset for s = |z|: j from y = s^2 by one multiply,
   clamped to jmax (NaN and inf clamp too), and d = s^2 - y_c with a single
   rounding (|d| <= h/2), so the full input precision reaches the
   polynomial, which matters because log R grows like y/(2 nu). */
__device__ __forceinline__ int cell_of(double s, double yh, int jmax, const StudentParams& P, double* d)
{
    double jd = yh * P.inv_h;
    const double jm = (double)jmax;
    jd = (jd < jm) ? jd : jm;
    int j = (int)jd;
    double yc = __builtin_fma((double)j, P.h, P.centre_offset);   /* exact: h is a power of 2 */
    *d = __builtin_fma(s, s, -yc);
    return j;
}

/* Beyond the LDS cells (y > y_lds, |z| above about 10).  Up to y_max the
   remaining cells, from global memory.  Beyond: w = K q(s),
   q(s) = erfcx(s/sqrt2) e^{-s^2/2} / 2, t = sqrt(nu) w^{-1/nu} (1 + a w^{2/nu})
   (Sections 3.3, 3.5), which the table builder has checked to be as accurate
   as the cells there.  log w is carried as a double-double (s^2/2 exactly,
   the division by nu with its remainder), because an absolute error e in it
   is a relative error e/nu in t and |log w| reaches several hundred. */
template <int DEG>
static __device__ __noinline__ double student_far(double s, const StudentParams& P)
{
#pragma clang fp contract(off)
    const double INV_SQRT2 = 0.70710678118654752440, LN2 = 0.69314718055994530942;
    if (!(s < __builtin_inf())) return s;              /* z = +-inf -> +-inf; NaN -> NaN */
    double yh = s * s;
    /* s^2 overflows (s above 1.3e154): log t is about s^2/(2 nu) > 700 for
       every nu below 1e300, so t overflows too */
    if (!(yh < __builtin_inf())) return yh;
    if (yh <= P.y_max) {
        double d;
        int j = cell_of(s, yh, P.ncell - 1, P, &d);
        return s * cell_poly<DEG>(P.gcoef + j * (DEG + 1), d);
    }
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

/* t(z) in FP64 from the LDS table, cells of degree DEG. */
template <int DEG>
__device__ __forceinline__ double student_eval(double z, const double* __restrict__ tab, const StudentParams& P)
{
    double s = __builtin_fabs(z);
    double yh = s * s;                      /* only selects the cell */
    double d;
    int j = cell_of(s, yh, P.nlds - 1, P, &d);
    double t = z * cell_poly_lds<DEG>(tab + j * P.lds_stride, d);
    bool far = !(yh <= P.y_lds);            /* also NaN: NaN propagates either way */
    if (wave_any(far)) {
        double tf = __builtin_copysign(student_far<DEG>(far ? s : 1.0, P), z);
        t = far ? tf : t;
    }
    return t;
}

}  // namespace qm

/*
 * qm_device.hpp -- per-element device math for gfx950 (wave64).
 *
 * Everything here is branch-free per lane.  The only control flow is
 * wave-uniform: a rare piece (the deep tail beyond the paper's v = 42) is
 * entered when any lane of the wave needs it, decided by a wave vote, so no
 * lane ever diverges from its neighbours (the paper's warp-vote idea,
 * Section 7.3, applied to the tail instead of the centre).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qm_coeffs.h"
#include "qm_paper_coeffs.h"

namespace qm {

/* Horner chain p <- p x + c, highest power first (Section 4.5.1: FMA-friendly
   iterated linear maps, no quadratic factorisation). */
template <int N>
__device__ __forceinline__ double horner(double x, const double (&c)[N])
{
    double acc = c[0];
#pragma unroll
    for (int i = 1; i < N; ++i) acc = __builtin_fma(acc, x, c[i]);
    return acc;
}

template <int N>
__device__ __forceinline__ float hornerf(float x, const float (&c)[N])
{
    float acc = c[0];
#pragma unroll
    for (int i = 1; i < N; ++i) acc = __builtin_fmaf(acc, x, c[i]);
    return acc;
}

/* FP32 Horner on FP64-stored coefficients (rounded once at compile time). */
template <int N>
__device__ __forceinline__ float hornerf_d(float x, const double (&c)[N])
{
    float acc = (float)c[0];
#pragma unroll
    for (int i = 1; i < N; ++i) acc = __builtin_fmaf(acc, x, (float)c[i]);
    return acc;
}

/* a / b for finite positive b of moderate size.  The hardware reciprocal is
   good to ~5e-8, so one Newton step on it (error ~2e-15) and one residual
   correction of the quotient give a result within an ulp. */
__device__ __forceinline__ double div_pos(double a, double b)
{
    double y = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(e, y, y);
    double q = a * y;
    double r = __builtin_fma(-b, q, a);
    return __builtin_fma(r, y, q);
}

/* sqrt(v) for positive normal v, within an ulp: hardware reciprocal square
   root (~5e-8), one coupled Newton step on (sqrt v, 1/(2 sqrt v)), one
   residual correction.  Other inputs give unspecified values. */
__device__ __forceinline__ double sqrt_pos(double v)
{
    double r = __builtin_amdgcn_rsq(v);
    double s = v * r, h = 0.5 * r;
    double e = __builtin_fma(-s, h, 0.5);
    s = __builtin_fma(s, e, s);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-s, s, v);
    return __builtin_fma(d, h, s);
}

/* -log(x) for x in (0, 1], relative error about an ulp.  x = m 2^e with m in
   [sqrt(1/2), sqrt(2)); log m = 2 atanh f = 2f + f s R(s), f = (m-1)/(m+1)
   (exact numerator), s = f^2, R a fitted degree-6 polynomial; log 2 is split
   so that e log2_hi is exact.  Denormal x is handled by frexp.  x = 0,
   negative or NaN x give unspecified values: callers select their results. */
__device__ __forceinline__ double neg_log_unit(double x)
{
    const double SQRT_HALF = 0.70710678118654752440;
    const double LN2_HI = 6.93147180369123816490e-01, LN2_LO = 1.90821492927058770002e-10;
    double m = __builtin_amdgcn_frexp_mant(x);
    int e = __builtin_amdgcn_frexp_exp(x);
    bool lo = m < SQRT_HALF;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    double f = div_pos(m - 1.0, m + 1.0);
    double s = f * f;
    double lm = __builtin_fma(f * s, horner(s, QM_LOG_R), f + f);
    double de = (double)e;
    return -__builtin_fma(de, LN2_HI, __builtin_fma(de, LN2_LO, lm));
}

/* any lane of the wave */
__device__ __forceinline__ bool wave_any(bool p) { return __any((int)p) != 0; }

/* ------------------------------------------------------------------------ */
/* Exponential-coordinate normal quantile Q(v) = Phi^{-1}(1 - e^{-v}/2),     */
/* v >= 0 (Section 6 formal solution; Section 7.2 branchless rational).      */
/* ------------------------------------------------------------------------ */

/* v > 750 (only reachable through exp -> normal with |x| > 750): from the
   Mills-ratio expansion of the normal tail, log q(z) = -z^2/2 - log(z sqrt(2 pi))
   + log S(z), S = 1 - z^-2 + 3 z^-4 - 15 z^-6 + 105 z^-8, solve
   z^2 = 2 (v + log 2 - log(z sqrt(2 pi)) + log S(z)) by fixed-point
   iteration; the map contracts by ~1/z^2 < 1/1500 per step. */
__device__ __noinline__ double expcoord_far(double v)
{
    const double LN2 = 0.69314718055994530942, LN_SQRT2PI = 0.91893853320467274178;
    double z = __builtin_sqrt(2.0) * __builtin_sqrt(v);
    for (int k = 0; k < 5; ++k) {
        double iz2 = 1.0 / (z * z);
        double S = __builtin_fma(__builtin_fma(__builtin_fma(105.0 * iz2 - 15.0, iz2, 3.0), iz2, -1.0), iz2, 1.0);
        double L = ::log(z) + LN_SQRT2PI - ::log(S);
        z = __builtin_sqrt(2.0) * __builtin_sqrt(v + (LN2 - L));
    }
    return z;
}

/*
 * Plain FP64 Q(v) for v in [0, inf]: the paper's (13,13) rational on
 * v <= 42 and the fitted Q(v) = s P7(s)/Q7(s), s = sqrt v, beyond.  Both
 * pieces end in a single division.  FAR enables the v > 750 piece.
 */
template <bool FAR>
__device__ __forceinline__ double expcoord_q_plain(double v)
{
    double num = v * horner(v, QM_PAPER_P13);
    double den = horner(v, QM_PAPER_Q13);
    bool tail = v > QM_TAIL_VMIN;
    if (wave_any(tail)) {
        double s = sqrt_pos(v);
        double nt = s * horner(s, QM_TAIL_P);
        double dt = horner(s, QM_TAIL_Q);
        num = tail ? nt : num;
        den = tail ? dt : den;
    }
    double q = div_pos(num, den);
    if (FAR) {
        bool far = (v > QM_TAIL_VMAX) && (v < __builtin_inf());
        if (wave_any(far)) {
            double f = expcoord_far(far ? v : 1000.0);
            q = far ? f : q;
        }
    }
    return q;
}

/* Paper mode: the (13,13) rational verbatim, whatever v (Appendix B). */
__device__ __forceinline__ double expcoord_q_paper(double v)
{
    return div_pos(v * horner(v, QM_PAPER_P13), horner(v, QM_PAPER_Q13));
}

/* ------------------------------------------------------------------------ */
/* FP64 normal quantile w(u) = Phi^{-1}(u).                                  */
/* ------------------------------------------------------------------------ */

/* Reflection x = 2 min(u, 1-u) is exact (1-u exact for u >= 1/2, Sterbenz);
   v = -log x; sign by u - 1/2 (+0 at u = 1/2).  u = 0 -> -inf, u = 1 -> +inf,
   u outside [0,1] or NaN -> NaN, all by select (Section 7.2 reflection; the
   paper's kernels leave u in {0,1} to NaN). */
__device__ __forceinline__ double quantile_v(double u)
{
    double om = 1.0 - u;
    double p = (u < om) ? u : om;
    return neg_log_unit(p + p);
}

__device__ __forceinline__ double quantile_finish(double u, double mag)
{
    double w = __builtin_copysign(mag, u - 0.5);
    w = (u == 0.0) ? -__builtin_inf() : w;
    w = (u == 1.0) ? __builtin_inf() : w;
    w = (u >= 0.0 && u <= 1.0) ? w : __builtin_nan("");
    return w;
}

/* The exponential-coordinate path for any u (plain mode): v = -log(2 min(u,
   1-u)), Q(v), sign and specials. */
__device__ __forceinline__ double outer_quantile_f64(double u)
{
    return quantile_finish(u, expcoord_q_plain<false>(quantile_v(u)));
}

/* Central piece, |q| <= 0.45 with q = u - 1/2 (90% of uniform draws):
   w = q P8(r)/Q8(r), r = 0.2025 - q^2, relative error 6e-17 after rounding;
   no logarithm.  q is exact for u >= 1/4 and within half an ulp below, which
   moves w by at most 2.3e-16 relative at |q| = 0.45.  Other q give
   unspecified values. */
__device__ __forceinline__ bool is_central(double q) { return __builtin_fabs(q) <= QM_CENTRAL_QMAX; }

__device__ __forceinline__ double central_quantile(double q)
{
    double r = __builtin_fma(-q, q, QM_CENTRAL_X);
    return div_pos(q * horner(r, QM_CENTRAL_P), horner(r, QM_CENTRAL_Q));
}

/*
 * FP64 w(u).  Paper mode: the (13,13) rational of Appendix B in the
 * exponential coordinate for every u.  Plain mode: the hybrid of
 * Section 7.3 / Appendix C -- a central piece where most samples fall, the
 * branchless exponential-coordinate path elsewhere -- with the paper's T2
 * central variable (chosen there for a fast single-precision-grade rsqrt)
 * replaced by q itself, which needs no transcendental at all.  Lanes
 * outside the centre take the outer path by wave vote here; the streaming
 * kernel instead gathers them across the wave (k_hybrid), with the
 * same arithmetic per element.
 */
template <bool PAPER>
__device__ __forceinline__ double normal_quantile_f64(double u)
{
    if (PAPER) return quantile_finish(u, expcoord_q_paper(quantile_v(u)));
    double q = u - 0.5;
    bool central = is_central(q);           /* NaN: false */
    double w = central_quantile(q);
    if (wave_any(!central)) {
        double wo = outer_quantile_f64(u);
        w = central ? w : wo;
    }
    return w;
}

/* 1/sqrt(x) for positive normal x, within about an ulp: the hardware
   reciprocal square root y (~5e-8), then y (1 + e/2 + 3e^2/8) with
   e = 1 - x y^2 (second-order Newton; e is exact up to the rounding of x y).
   Zero, denormal, negative or NaN x give values that callers must not use. */
__device__ __forceinline__ double rsqrt_pos(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    double e = __builtin_fma(-h, y, 1.0);
    double c = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y * e, c, y);
}

/*
 * The paper's own FP64 hybrid (Section 7.3, Appendix C), constants as
 * printed.  Every lane forms the T2 coordinate v = |u - 1/2| / sqrt(u(1-u));
 * if v < 15.5 on every lane of the wave, the wave takes Psi(v) = v P14/Q15,
 * otherwise the whole wave takes the branchless (13,13) path of Appendix B.
 * u(1-u) is formed as a product rather than the printed u - u*u, which
 * cancels near u = 1 (relative error up to 5e-14 at u = 0.999 there, 1.5
 * ulp here).  u = 1/2 -> +0; u = 0, 1, NaN or outside [0,1] give v >= 15.5
 * or NaN, so the branchless path's specials apply.
 */
__device__ __forceinline__ double t2_coord(double u, double& q)
{
    q = u - 0.5;
    return __builtin_fabs(q) * rsqrt_pos(u * (1.0 - u));
}

__device__ __forceinline__ double t2_psi(double v, double q)
{
    return __builtin_copysign(div_pos(v * horner(v, QM_PAPER_T2_P14), horner(v, QM_PAPER_T2_Q15)), q);
}

__device__ __forceinline__ double normal_quantile_f64_t2(double u)
{
    double q;
    double v = t2_coord(u, q);
    if (__all((int)(v < QM_PAPER_T2_VMAX))) return t2_psi(v, q);
    return quantile_finish(u, expcoord_q_paper(quantile_v(u)));
}

/* Exponential -> normal, FP64: v = |x| directly, odd extension. */
template <bool PAPER>
__device__ __forceinline__ double exp_to_normal_f64(double x)
{
    double v = __builtin_fabs(x);
    double mag = PAPER ? expcoord_q_paper(v) : expcoord_q_plain<true>(v);
    mag = (v == __builtin_inf()) ? v : mag;
    return __builtin_copysign(mag, x);
}

/* ------------------------------------------------------------------------ */
/* FP32 + FP64-refine form.                                                  */
/* ------------------------------------------------------------------------ */

/* -log(x) for x in (0, 1] in FP32 with the hardware log2, denormals scaled
   into the normal range first (accuracy is only needed at the seed level). */
__device__ __forceinline__ float neg_log_f32(float x)
{
    const float LN2F = 0.693147180559945309f;
    bool sub = x < 0x1p-126f;
    float xs = sub ? x * 0x1p32f : x;
    float l2 = __builtin_amdgcn_logf(xs);          /* v_log_f32: log2 */
    return __builtin_fmaf(-l2, LN2F, sub ? 32.0f * LN2F : 0.0f);
}

/* FP32 seed of Q(v) = v P4(v)/Q5(v), relative error ~1.2e-5 on v <= 103.3 */
__device__ __forceinline__ float expcoord_seed_f32(float v)
{
    float num = v * hornerf_d(v, QM_SEED_P);
    float den = hornerf_d(v, QM_SEED_Q);
    return num * __builtin_amdgcn_rcpf(den);
}

/* e^a for |a| <= 700 for the correction steps: a = k ln2 + r,
   |r| <= ln2/2, the degree-DEG Taylor polynomial in r, then scale by 2^k.
   Relative error below the remainder (ln2/2)^(DEG+1)/(DEG+1)!: 7e-12 for
   degree 9, 5.3e-9 for degree 7. */
template <int DEG>
__device__ __forceinline__ double exp_refine(double a)
{
    const double LOG2E = 1.4426950408889634074, LN2_HI = 0.69314718055994528623, LN2_LO = 2.3190468138462996154e-17;
    double k = __builtin_rint(a * LOG2E);
    double r = __builtin_fma(-k, LN2_HI, a);
    r = __builtin_fma(-k, LN2_LO, r);
    double f = 1.0;
#pragma unroll
    for (int i = 2; i <= DEG; ++i) f *= i;           /* DEG!, folded at compile time */
    double p = 1.0 / f;
#pragma unroll
    for (int i = DEG; i >= 1; --i) {
        f /= i;                                       /* (i-1)! */
        p = __builtin_fma(p, r, 1.0 / f);
    }
    return __builtin_ldexp(p, (int)k);
}

/* a / b to ~3e-15 for positive b of moderate size: hardware reciprocal and
   one Newton step, no residual correction (enough for the correction step's
   1e-11 needs). */
__device__ __forceinline__ double div_pos_fast(double a, double b)
{
    double y = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, y, 1.0);
    y = __builtin_fma(e, y, y);
    return a * y;
}

/*
 * One Halley correction of x0 ~ z >= 0 solving q(z) = p, q(z) = 1 - Phi(z),
 * against an FP64 erfc written as erfc(z/sqrt2) = 2 phi(z) M(z) with the
 * Mills ratio M from a fitted rational (relative 1.1e-12 on [0, 14.5]).
 * With G(x) = q(x) - p = phi(x) t, t = M(x) - p/phi(x), G' = -phi, G'' = x phi:
 *   Halley:  x1 = x0 + t / (1 - x0 t / 2) ~ x0 + t (1 + x0 t / 2)
 * (the expansion drops O(x0^2 t^3), below 1e-10 relative for a 1e-5 seed).
 * The caller supplies p/phi(x0), formed so that it stays in range.
 */
template <int NP, int NQ>
__device__ __forceinline__ double halley_upper(double x0, double p_over_phi, const double (&MP)[NP],
                                               const double (&MQ)[NQ])
{
    double M = div_pos_fast(horner(x0, MP), horner(x0, MQ));
    double t = M - p_over_phi;
    double h = 0.5 * x0 * t;
    return __builtin_fma(t, 1.0 + h, x0);
}

/* One Newton correction of x0 ~ z >= 0 solving q(z) = p (notation as for
 * halley_upper): x1 = x0 + t.  Newton leaves (x0/2) e0^2 of a seed error e0,
 * i.e. x0^2 eps^2 / 2 relative for a relative seed error eps: 1.4e-8 at
 * z = 14 for the 1.2e-5 seed below, so Halley's extra factor is not needed
 * there. */
template <int NP, int NQ>
__device__ __forceinline__ double newton_upper(double x0, double p_over_phi, const double (&MP)[NP],
                                               const double (&MQ)[NQ])
{
    double t = div_pos_fast(horner(x0, MP), horner(x0, MQ)) - p_over_phi;
    return x0 + t;
}

/* Phi^{-1}(u) for FP32 u outside the centre: FP32 seed in the exponential
   coordinate (1.2e-5) + one FP64 Newton step, rounded to FP32.  Here
   z > 1.6449, so the step takes the Mills ratio of [1.6, 14.5] (8.5e-9,
   moving the result by about 8.5e-9 / z^2 relative) and the degree-7
   exponential (5.3e-9, by about 5.3e-9 / z^2). */
__device__ __forceinline__ float outer_quantile_f32_refine(float u)
{
    const double SQRT2PI = 2.5066282746310005024;
    float om = 1.0f - u;                       /* exact for u >= 1/2 */
    float p = (u < om) ? u : om;
    float v = neg_log_f32(p + p);
    float z0 = expcoord_seed_f32(v);
    double x0 = (double)z0;
    double pd = (double)p;
    /* x0 has a 24-bit significand, so x0*x0/2 is exact in FP64 */
    double p_over_phi = pd * SQRT2PI * exp_refine<7>(0.5 * (x0 * x0));
    double x1 = newton_upper(x0, p_over_phi, QM_MILLS32_P, QM_MILLS32_Q);
    /* u = 0 and u = 1 both give p = 0: +-inf by the sign of u - 1/2 */
    float mag = (p == 0.0f) ? __builtin_inff() : (float)x1;
    /* NaN and out-of-range inputs need no select: p + p is then negative or
       NaN, the hardware log returns NaN, and NaN propagates to the result */
    return __builtin_copysignf(mag, u - 0.5f);
}

/*
 * Central piece of the FP32+refine form, |q| <= 0.45, q = u - 1/2 (qd, exact
 * in FP64 for FP32 u; qf, its FP32 value, serves the seed only): the FP32
 * seed z0 = q S2(r)/S3(r), r = 0.2025 - q^2 (2.6e-6 relative), then one
 * FP64 Newton step on Phi(z) = u,
 *   z1 = z0 - (erf(z0/sqrt2)/2 - q) / phi(z0),
 * with erf(z/sqrt2)/2 = z E6(z^2) (9.2e-9) and 1/phi(z) = G3(z^2) (1.1e-3).
 * E's error reaches z1 divided by phi(z) (at most 2.7 x 9.2e-9 relative, at
 * |q| = 0.45); G's only scales the step, about 2.6e-6 z, so it costs 2.9e-9
 * z; Newton's own error is (z0/2) e0^2, below 1e-11 z.  About 3e-8 in all,
 * before the rounding to FP32.  No logarithm and no exponential.
 */
__device__ __forceinline__ float central_quantile_f32_refine(float qf, double qd)
{
    float rf = __builtin_fmaf(-qf, qf, (float)QM_CENTRAL_X);
    float z0 = qf * hornerf_d(rf, QM_C32_SP) * __builtin_amdgcn_rcpf(hornerf_d(rf, QM_C32_SQ));
    double x0 = (double)z0;
    double y = x0 * x0;
    double res = __builtin_fma(x0, horner(y, QM_C32_E), -qd);
    return (float)__builtin_fma(-res, horner(y, QM_C32_G), x0);
}

/* Phi^{-1}(u) for FP32 u, FP32+refine form: the hybrid of the FP64 path
   (central piece; the outer path by wave vote here, gathered across the
   wave by the streaming kernel, with the same arithmetic per element). */
__device__ __forceinline__ float normal_quantile_f32_refine(float u)
{
    double qd = (double)u - 0.5;
    bool central = is_central(qd);          /* NaN: false */
    float w = central_quantile_f32_refine(u - 0.5f, qd);
    if (wave_any(!central)) {
        float wo = outer_quantile_f32_refine(u);
        w = central ? w : wo;
    }
    return w;
}

/* Phi^{-1}(u), FP32 u, paper's (5,6) in FP32 verbatim (Appendix A), with the
   specials fixed as above. */
__device__ __forceinline__ float normal_quantile_f32_paper(float u)
{
    float om = 1.0f - u;
    float p = (u < om) ? u : om;
    float v = neg_log_f32(p + p);
    float mag = v * hornerf(v, QM_PAPER_P5) * __builtin_amdgcn_rcpf(hornerf(v, QM_PAPER_Q6));
    float w = __builtin_copysignf(mag, u - 0.5f);
    w = (u == 0.0f) ? -__builtin_inff() : w;
    w = (u == 1.0f) ? __builtin_inff() : w;
    w = (u >= 0.0f && u <= 1.0f) ? w : __builtin_nanf("");
    return w;
}

/* Phi^{-1}(u), FP32 u, evaluated by the plain FP64 path and rounded. */
__device__ __forceinline__ float normal_quantile_f32_plain(float u)
{
    return (float)normal_quantile_f64<false>((double)u);
}

/* |x| > 103 for the FP32 form: the plain FP64 map, rounded (kept out of line:
   it is rare and would otherwise crowd the FP32 loop's registers). */
__device__ __noinline__ float exp_to_normal_f32_big(float v)
{
    float mb = (float)expcoord_q_plain<true>((double)v);
    return (v == __builtin_inff()) ? v : mb;
}

/* Exponential -> normal for FP32 x: FP32 seed Q(|x|) then one FP64 Halley
   step against q(z) = e^{-|x|}/2, for which
   p/phi(x0) = sqrt(pi/2) e^{x0^2/2 - |x|}; the exponent is O(log |x|).
   |x| > 103 (beyond the seed's fit) takes the plain FP64 path, by wave vote. */
__device__ __forceinline__ float exp_to_normal_f32_refine(float x)
{
    const double SQRT_HALF_PI = 1.2533141373155002512;
    float v = __builtin_fabsf(x);
    bool big = !(v <= 103.0f);                  /* also inf and NaN */
    float vs = big ? 1.0f : v;
    double x0 = (double)expcoord_seed_f32(vs);
    double a = __builtin_fma(0.5 * x0, x0, -(double)vs);
    double x1 = halley_upper(x0, SQRT_HALF_PI * exp_refine<9>(a), QM_MILLS_P, QM_MILLS_Q);
    float mag = (float)x1;
    mag = (vs == 0.0f) ? 0.0f : mag;
    if (wave_any(big)) {
        float mb = exp_to_normal_f32_big(v);
        mag = big ? mb : mag;
    }
    return __builtin_copysignf(mag, x);
}

}  // namespace qm

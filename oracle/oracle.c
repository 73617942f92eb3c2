/*
 * oracle.c -- slow, plain CPU reference for the quantile-mechanics hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may use it.  It shares no code, header, table or constant
 * with the GPU library; the only thing both sides share is the seeded input
 * generator (qm_inputs/), which holds none of the method's arithmetic.
 *
 * What is computed (Shaw, Luu & Brickman, "Quantile Mechanics II"):
 *
 *   norm_quantile   w(u) = Phi^{-1}(u), the quantile defined by F(w(u)) = u
 *                   (Section 1, eqs. 1-2) for the standard normal F = Phi.
 *   exp_to_normal   Q(x) = sign(x) Phi^{-1}(1 - exp(-|x|)/2), the formal
 *                   solution of the exponential-background recycling ODE with
 *                   Q(0) = 0, Q'(0) = sqrt(pi/2), extended to x < 0 by odd
 *                   symmetry (Section 6).
 *   student_t_map   Q(z) = F_nu^{-1}(Phi(z)), the recycling map from a normal
 *                   sample to a Student t sample with nu (real, > 0) degrees of
 *                   freedom (Section 1 recycling composite; Section 3.1).
 *
 * Each is computed from its plain definition: the target CDF is evaluated in
 * x87 extended precision (64-bit significand) and the defining equation is
 * solved for the FP64 result, which is then checked against its two FP64
 * neighbours so that the returned double is the one with the smallest
 * residual.  No approximation from the paper is used here; the paper's
 * rationals and series only appear in the tests, as independent pins.
 *
 * Error behaviour: per-element, never an error code.  NaN in -> NaN out,
 * u outside [0,1] -> NaN, u = 0 -> -inf, u = 1 -> +inf.
 */
#include <math.h>
#include <float.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <pthread.h>
#include <unistd.h>

typedef long double ld;

#define LD_SQRT2   1.41421356237309504880168872420969808L
#define LD_SQRT2PI 2.50662827463100050241576528481104525L
#define LD_LN2     0.693147180559945309417232121458176568L

/* ------------------------------------------------------------------------- */
/* Standard normal tail probability q(z) = 1 - Phi(z) = erfc(z/sqrt2)/2 and   */
/* its logarithm.  erfcl underflows near z ~ 150; beyond z = 35 the log is   */
/* taken from the asymptotic expansion of the Mills ratio,                  */
/*   q(z) = phi(z)/z * (1 - 1/z^2 + 3/z^4 - 15/z^6 + ...),                   */
/* whose terms at z >= 35 fall below 1e-24 after a dozen terms.              */
/* ------------------------------------------------------------------------- */
static ld norm_upper(ld z) { return 0.5L * erfcl(z / LD_SQRT2); }

static ld log_norm_upper(ld z)
{
    if (z < 35.0L) return logl(norm_upper(z));
    ld iz2 = 1.0L / (z * z), term = 1.0L, sum = 1.0L;
    for (int k = 1; k < 40; ++k) {
        term *= -(ld)(2 * k - 1) * iz2;
        sum += term;
        if (fabsl(term) < 1e-30L) break;
    }
    return -0.5L * z * z - logl(z * LD_SQRT2PI) + logl(sum);
}

static ld norm_pdf(ld z) { return expl(-0.5L * z * z) / LD_SQRT2PI; }

/* ------------------------------------------------------------------------- */
/* Safeguarded Newton on a monotone scalar equation g(z) = 0 over [lo, hi].   */
/* The bracket is kept; a Newton step that leaves it, or that fails to halve  */
/* the residual, is replaced by bisection.                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int kind;  /* 0: erf(z/sqrt2) - r ; 1: log q(z) - logp */
    ld r;      /* target of kind 0 */
    ld logp;   /* target of kind 1 */
} norm_eq;

static ld norm_eq_g(const norm_eq* e, ld z)
{
    if (e->kind == 0) return erfl(z / LD_SQRT2) - e->r;
    return log_norm_upper(z) - e->logp;
}

/* derivative dg/dz */
static ld norm_eq_dg(const norm_eq* e, ld z)
{
    if (e->kind == 0) return 2.0L * norm_pdf(z);
    /* d/dz log q(z) = -phi(z)/q(z) = -1/M(z); evaluate in log form so that it
       stays finite where q and phi both underflow */
    ld lq = log_norm_upper(z);
    ld lphi = -0.5L * z * z - logl(LD_SQRT2PI);
    return -expl(lphi - lq);
}

/* Solve for z >= 0; g increasing (kind 0) or decreasing (kind 1). */
static ld newton_bracketed(const norm_eq* e, ld lo, ld hi, ld z)
{
    ld glo = norm_eq_g(e, lo);
    ld gprev = INFINITY;
    for (int it = 0; it < 400; ++it) {
        ld g = norm_eq_g(e, z);
        if (g == 0.0L) return z;
        if ((g > 0) == (glo > 0)) { lo = z; glo = g; } else { hi = z; }
        ld d = norm_eq_dg(e, z);
        ld zn = z - g / d;
        int bad = !(zn > lo && zn < hi) || !(fabsl(g) <= 0.5L * fabsl(gprev)) || !isfinite(zn);
        if (bad && it > 0) zn = 0.5L * (lo + hi);
        if (!(zn > lo && zn < hi)) zn = 0.5L * (lo + hi);
        gprev = g;
        /* converged to a few units of the extended-precision significand */
        if (fabsl(zn - z) <= 8.0L * LDBL_EPSILON * fabsl(z) || hi - lo <= 8.0L * LDBL_EPSILON * fabsl(hi))
            return zn;
        z = zn;
    }
    return z;
}

/* Pick the double nearest in residual among round(z) and its neighbours. */
static double best_double(const norm_eq* e, ld z)
{
    double d = (double)z;
    double c[3] = { nextafter(d, -INFINITY), d, nextafter(d, INFINITY) };
    double best = d;
    ld bres = INFINITY;
    for (int i = 0; i < 3; ++i) {
        if (c[i] < 0.0) continue;
        ld r = fabsl(norm_eq_g(e, (ld)c[i]));
        if (r < bres) { bres = r; best = c[i]; }
    }
    return best;
}

/* z >= 0 with q(z) = p, for p in (0, 1/2].  (Section 1, eq. 1 with F = Phi.) */
static double upper_quantile(double p)
{
    norm_eq e;
    if (p >= 0.25) {
        /* erf(z/sqrt2) = 1 - 2p; the right-hand side is exact in FP64 here
           (Sterbenz), so the solve is relative-accurate as z -> 0. */
        e.kind = 0;
        e.r = (ld)(1.0 - 2.0 * p);
        if (e.r == 0.0L) return 0.0;
        ld z0 = e.r * 1.2533141373155002512L;   /* slope of Phi^{-1} at 1/2 */
        if (z0 > 0.7L) z0 = 0.35L;
        return best_double(&e, newton_bracketed(&e, 0.0L, 0.7L, z0));
    }
    e.kind = 1;
    e.logp = logl((ld)p);
    ld z0 = sqrtl(-2.0L * e.logp);
    if (z0 > 39.0L) z0 = 39.0L;
    if (z0 < 0.7L) z0 = 0.7L;
    return best_double(&e, newton_bracketed(&e, 0.6L, 40.0L, z0));
}

double oracle_norm_quantile1(double u)
{
    if (isnan(u) || u < 0.0 || u > 1.0) return NAN;
    if (u == 0.0) return -INFINITY;
    if (u == 1.0) return INFINITY;
    if (u == 0.5) return 0.0;
    if (u < 0.5) return -upper_quantile(u);
    return upper_quantile(1.0 - u);   /* 1 - u exact for u >= 1/2 */
}

/* ------------------------------------------------------------------------- */
/* Exponential -> normal (Section 6): Q(x) = Phi^{-1}(1 - e^{-x}/2), x >= 0,  */
/* i.e. q(Q) = e^{-x}/2, extended by odd symmetry.  For x >= ln 2 the        */
/* equation is solved in log space, log q(z) = -x - ln 2; below ln 2 it is   */
/* solved as erf(z/sqrt2) = 1 - e^{-x} = -expm1(-x), which stays relative-   */
/* accurate as x -> 0.                                                       */
/* ------------------------------------------------------------------------- */
double oracle_exp_to_normal1(double x)
{
    if (isnan(x)) return NAN;
    if (x == 0.0) return x;
    if (isinf(x)) return x;
    ld a = fabsl((ld)x);
    norm_eq e;
    double z;
    if (a < LD_LN2) {
        e.kind = 0;
        e.r = -expm1l(-a);
        ld z0 = a * 1.2533141373155002512L;
        if (z0 > 0.7L) z0 = 0.35L;
        z = best_double(&e, newton_bracketed(&e, 0.0L, 0.7L, z0));
    } else {
        e.kind = 1;
        e.logp = -a - LD_LN2;
        ld hi = sqrtl(2.0L * a + 8.0L) + 2.0L;   /* q(hi) < e^{-a}/2 */
        ld z0 = sqrtl(2.0L * a);
        if (z0 < 0.6L) z0 = 0.6L;
        if (z0 > hi) z0 = 0.5L * hi;
        z = best_double(&e, newton_bracketed(&e, 0.6L, hi, z0));
    }
    return x < 0 ? -z : z;
}

/* ------------------------------------------------------------------------- */
/* Student t (Section 3.1 density).  CDF through the regularized incomplete  */
/* beta function: for t >= 0,                                                */
/*   1 - F_nu(t) = I_{nu/(nu+t^2)}(nu/2, 1/2) / 2,                            */
/*   F_nu(t) - 1/2 = I_{t^2/(nu+t^2)}(1/2, nu/2) / 2.                          */
/* I_x(a,b) is evaluated from its continued fraction (DLMF 8.17.22) with the */
/* modified Lentz method where x < (a+1)/(a+b+2), else through the symmetry  */
/* I_x(a,b) = 1 - I_{1-x}(b,a) (DLMF 8.17.4).  Both x and 1-x, and their     */
/* logarithms, are passed in so that none is formed by cancellation: with    */
/* x = nu/(nu+t^2), log x = -log1p(t^2/nu), since the prefactor raises x to  */
/* the power nu/2 and would multiply a rounding of x by nu/2.                */
/* ------------------------------------------------------------------------- */
static ld lbeta(ld a, ld b) { return lgammal(a) + lgammal(b) - lgammal(a + b); }

/*
 * log B(a, 1/2) = log Gamma(1/2) - D(a), D(a) = log Gamma(a+1/2) - log Gamma(a).
 * For large a the difference of two lgamma values near a log a would lose
 * its last digits times a log a; instead a = r + k with r in [1, 2) and, by
 * Gamma(x+1) = x Gamma(x) (DLMF 5.5.1),
 *   D(a) = D(r) + sum_{j<k} log(1 + 1/(2(r+j))),
 * summed with compensation (Kahan).
 */
static ld lbeta_half(ld a)
{
    if (a < 16.0L) return lbeta(a, 0.5L);
    ld k = floorl(a) - 1.0L, r = a - k;
    ld sum = lgammal(r + 0.5L) - lgammal(r), comp = 0.0L;
    for (ld j = 0.0L; j < k; j += 1.0L) {
        ld term = log1pl(0.5L / (r + j)) - comp;
        ld t = sum + term;
        comp = (t - sum) - term;
        sum = t;
    }
    return lgammal(0.5L) - sum;
}

/*
 * K = 1 + d1/(1 + d2/(1 + ...)), so that I_x(a,b) = prefactor / K, with the
 * partial numerators d_j of DLMF 8.17.22.  For large a near the switch point
 * d1 = -(a+b)x/(a+1) is close to -1 and K ~ 1/a: forming 1 + d1/T (T the
 * rest of the fraction) would lose the digits of K.  So c1 = 1 + d1 =
 * ((a+1)(1-x) + (1-b)x)/(a+1) is formed directly from 1-x, the rest
 * R = T - 1 = d2/(1 + d3/(1 + ...)) by the modified Lentz method, and
 * K = (c1 + R)/(1 + R).
 */
static ld beta_cf(ld a, ld b, ld x, ld omx)
{
    const ld tiny = 1e-4000L, eps = 1e-21L;
    ld f = tiny, C = tiny, D = 0.0L;
    for (int j = 2; j < 40000; ++j) {
        int m = j / 2;
        ld dj;
        if (j & 1) dj = -(a + m) * (a + b + m) * x / ((a + 2 * m) * (a + 2 * m + 1));
        else       dj = m * (b - m) * x / ((a + 2 * m - 1) * (a + 2 * m));
        D = 1.0L + dj * D;
        if (fabsl(D) < tiny) D = tiny;
        C = 1.0L + dj / C;
        if (fabsl(C) < tiny) C = tiny;
        D = 1.0L / D;
        ld delta = C * D;
        f *= delta;
        if (fabsl(delta - 1.0L) < eps) break;
    }
    ld c1 = ((a + 1.0L) * omx + (1.0L - b) * x) / (a + 1.0L);
    return (c1 + f) / (1.0L + f);
}

/* x^a (1-x)^b / (a B(a,b)) from lx = log x, lomx = log(1-x), lb = log B */
static ld beta_prefactor(ld a, ld b, ld lx, ld lomx, ld lb)
{
    return expl(a * lx + b * lomx - lb) / a;
}

/* I_x(a,b) with omx = 1 - x, lx = log x, lomx = log(1-x); lbab = log B(a,b)
   (symmetric in a,b). */
static ld betainc_reg(ld a, ld b, ld x, ld omx, ld lx, ld lomx, ld lbab)
{
    if (x <= 0.0L) return 0.0L;
    if (omx <= 0.0L) return 1.0L;
    if (x < (a + 1.0L) / (a + b + 2.0L))
        return beta_prefactor(a, b, lx, lomx, lbab) / beta_cf(a, b, x, omx);
    return 1.0L - beta_prefactor(b, a, lomx, lx, lbab) / beta_cf(b, a, omx, x);
}

double oracle_betainc(double a, double b, double x)
{
    if (!(a > 0) || !(b > 0) || !(x >= 0) || !(x <= 1)) return NAN;
    return (double)betainc_reg(a, b, x, 1.0L - (ld)x, logl(x), log1pl(-(ld)x), lbeta(a, b));
}

/* 1 - F_nu(t) for t >= 0, and F_nu(t) - 1/2 for t >= 0 */
typedef struct { ld nu, lb; } tctx;

/* with s = t^2/nu: log(nu/(nu+t^2)) = -log1p(s), log(t^2/(nu+t^2)) = -log1p(1/s) */
static ld t_upper(const tctx* c, ld t)
{
    ld t2 = t * t;
    ld x = c->nu / (c->nu + t2), omx = t2 / (c->nu + t2);
    ld lx = -log1pl(t2 / c->nu), lomx = -log1pl(c->nu / t2);
    return 0.5L * betainc_reg(0.5L * c->nu, 0.5L, x, omx, lx, lomx, c->lb);
}

static ld t_central(const tctx* c, ld t)
{
    ld t2 = t * t;
    ld y = t2 / (c->nu + t2), omy = c->nu / (c->nu + t2);
    ld ly = -log1pl(c->nu / t2), lomy = -log1pl(t2 / c->nu);
    return 0.5L * betainc_reg(0.5L, 0.5L * c->nu, y, omy, ly, lomy, c->lb);
}

static uint64_t dbits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }
static double bitsd(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }

/*
 * Q(z) = F_nu^{-1}(Phi(z)) by bisection over the IEEE-754 bit pattern of
 * t >= 0 (the bit pattern of non-negative doubles is monotone in the value),
 * ending on two adjacent doubles; the one with the smaller residual wins.
 */
static double student_map1(const tctx* c, double z)
{
    if (isnan(z)) return NAN;
    if (z == 0.0) return z;
    if (isinf(z)) return z;
    ld s = fabsl((ld)z);
    /* below s = 0.67, Phi(s) - 1/2 < 1/4: solve the central form */
    int central = (s <= 0.67L);
    ld target = central ? 0.5L * erfl(s / LD_SQRT2) : norm_upper(s);
    if (!central && s >= 35.0L) target = expl(log_norm_upper(s));
    /* residual, oriented to increase with t */
    #define RES(tv) (central ? (t_central(c, (ld)(tv)) - target) : (target - t_upper(c, (ld)(tv))))
    uint64_t lo = 0, hi = dbits(DBL_MAX);
    if (RES(DBL_MAX) < 0.0L) return z < 0 ? -INFINITY : INFINITY;
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (RES(bitsd(mid)) < 0.0L) lo = mid; else hi = mid;
    }
    double tl = bitsd(lo), th = bitsd(hi);
    ld rl = fabsl(RES(tl)), rh = fabsl(RES(th));
    #undef RES
    double t = (rl < rh) ? tl : th;
    return z < 0 ? -t : t;
}

double oracle_student_t_map1(double z, double nu)
{
    if (isnan(nu) || !(nu > 0.0)) return NAN;
    if (isinf(nu)) return z;
    tctx c = { (ld)nu, lbeta_half(0.5L * (ld)nu) };
    return student_map1(&c, z);
}

/* ------------------------------------------------------------------------- */
/* Array drivers, split over threads (nthreads <= 0: all online cores).       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int op;              /* 0 norm_quantile, 1 exp_to_normal, 2 student */
    const double* in;
    double* out;
    size_t begin, end;
    double nu;
} job;

static void* run_job(void* p)
{
    job* j = (job*)p;
    if (j->op == 2) {
        if (isnan(j->nu) || !(j->nu > 0.0)) {
            for (size_t i = j->begin; i < j->end; ++i) j->out[i] = NAN;
            return NULL;
        }
        if (isinf(j->nu)) {
            for (size_t i = j->begin; i < j->end; ++i) j->out[i] = j->in[i];
            return NULL;
        }
        tctx c = { (ld)j->nu, lbeta_half(0.5L * (ld)j->nu) };
        for (size_t i = j->begin; i < j->end; ++i) j->out[i] = student_map1(&c, j->in[i]);
        return NULL;
    }
    for (size_t i = j->begin; i < j->end; ++i)
        j->out[i] = (j->op == 0) ? oracle_norm_quantile1(j->in[i]) : oracle_exp_to_normal1(j->in[i]);
    return NULL;
}

static int run_parallel(int op, const double* in, double* out, size_t n, double nu, int nthreads)
{
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((size_t)nthreads > n) nthreads = n ? (int)n : 1;
    pthread_t th[256];
    int joined[256];
    job jobs[256];
    size_t per = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        size_t b = (size_t)t * per, e = b + per;
        if (b > n) b = n;
        if (e > n) e = n;
        jobs[t] = (job){ op, in, out, b, e, nu };
        joined[t] = 0;
        if (nthreads == 1 || pthread_create(&th[t], NULL, run_job, &jobs[t]) != 0) {
            run_job(&jobs[t]);   /* run inline when no thread could be started */
            continue;
        }
        joined[t] = 1;
    }
    for (int t = 0; t < nthreads; ++t)
        if (joined[t]) pthread_join(th[t], NULL);
    return nthreads;
}

int oracle_norm_quantile(const double* u, double* w, size_t n, int nthreads)
{ return run_parallel(0, u, w, n, 0.0, nthreads); }

int oracle_exp_to_normal(const double* x, double* z, size_t n, int nthreads)
{ return run_parallel(1, x, z, n, 0.0, nthreads); }

int oracle_student_t_map(const double* z, double* t, size_t n, double nu, int nthreads)
{ return run_parallel(2, z, t, n, nu, nthreads); }

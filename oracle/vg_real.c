/*
 * vg_real.c -- oracle for the exponential -> variance-gamma recycling map
 * with real lambda >= 1.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c and vg.c: nothing in the product
 * library calls, links or loads this file, and it shares no code with it.
 *
 * What is computed (Shaw, Luu & Brickman, "Quantile Mechanics II", Section
 * 8.2).  Target: the variance-gamma density (mu = 0)
 *     f(x) = A e^{beta x} |x|^{nu} K_nu(alpha |x|),   nu = lambda - 1/2,
 *     A = (alpha^2 - beta^2)^lambda / ((2 alpha)^nu sqrt(pi) Gamma(lambda)),
 * lambda > 0, |beta| < alpha.  Base and map as for the hyperbolic target
 * (Section 8.1): the two-sided exponential base with the target's masses
 * p+, p- and rates alpha - beta (v >= 0), alpha + beta (v < 0);
 * 1 - F(Q) = p+ e^{-(alpha - beta) v} for v >= 0, the mirror image
 * (beta -> -beta) for v < 0.
 *
 * Method, written from the definitions rather than from the recycling ODE
 * (the product's route), and unlike vg.c valid for any real lambda:
 * with the integral K_nu(z) = int_0^inf e^{-z cosh s} cosh(nu s) ds
 * (DLMF 10.32.9) and the order of integration exchanged (all terms
 * positive), each side's masses become one integral over s,
 *     T(x) = int_x^inf f = A int_0^inf cosh(nu s) c(s)^{-a} Gamma(a, c(s) x) ds,
 *     M(x) = int_0^x  f = A int_0^inf cosh(nu s) c(s)^{-a} gamma(a, c(s) x) ds,
 * c(s) = alpha cosh s - beta > 0, a = lambda + 1/2, with the upper and lower
 * incomplete gamma functions of real order a.  The s-integrand is even and
 * analytic in the strip |Im s| < arccos(beta/alpha) (where c vanishes), so
 * the trapezoidal rule on [0, inf) with half weight at 0 converges like
 * e^{-2 pi d / h}; h = d/10 puts that below 1e-27.  Summation stops once the
 * terms have fallen below 1e-23 of the sum for good.  (Far from the real
 * axis, beta < 0 makes Re c(s) negative beyond |Im s| = pi/2, where the
 * e^{-c x} of the incomplete gamma grows, so d is capped at pi/2, and
 * h = d/10; far out, where e^{-c x} off the axis outgrows its value on the
 * axis, h also shrinks like 1/sqrt(alpha x).)  gamma(a, y) is the
 * power series y^a e^{-y} sum_k y^k / (a (a+1) ... (a+k)) (DLMF 8.7.1 in the
 * form of Temme's series) for y < a + 1, and Gamma(a, y) the continued
 * fraction of Legendre (DLMF 8.9.2) by the modified Lentz method beyond;
 * each is completed from the other with Gamma(a) where needed.  Far out the
 * upper tail is summed with e^{-(alpha - beta) x} and the power y^{a-1}
 * taken out, in logarithms, so nothing underflows.
 *
 * The map is solved like the other oracles: bisection over the IEEE-754
 * bit pattern of x >= 0, central form M(x) = p+ (1 - e^{-r v}) while
 * r v <= ln 2, log tail log T(x) = log p+ - r v beyond, ending on two
 * adjacent doubles; the one with the smaller residual is returned.  Long
 * double throughout.
 *
 * Error behaviour: per element; NaN -> NaN, +-inf -> +-inf; parameters
 * outside lambda in [1, 64], alpha > |beta|, all finite -> NaN.
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

typedef long double ld;

static const ld LN2L = 0.693147180559945309417232121458176568L;
static const ld PIL = 3.141592653589793238462643383279502884L;

/* ---- incomplete gamma functions of real order a > 0, y >= 0 ---- */

/* gamma(a, y) e^{y} y^{-a} = sum_k y^k / (a (a+1) ... (a+k)) */
static ld lower_series(ld a, ld y)
{
    ld term = 1 / a, sum = term;
    for (int k = 1; k < 100000; ++k) {
        term *= y / (a + k);
        sum += term;
        if (term <= 1e-22L * sum) break;
    }
    return sum;
}

/* Gamma(a, y) e^{y} y^{1-a} by Legendre's continued fraction
   Gamma(a, y) = e^{-y} y^a / (y + 1 - a - 1 (1 - a)/(y + 3 - a - 2 (2 - a)/(y + 5 - a - ...))),
   evaluated by the modified Lentz method; y >= a + 1 */
static ld upper_cf(ld a, ld y)
{
    const ld tiny = 1e-4000L;
    ld b = y + 1 - a;
    ld c = 1 / tiny, d = 1 / b, h = d;
    for (int k = 1; k < 100000; ++k) {
        ld an = -k * (k - a);
        b += 2;
        d = an * d + b;
        if (fabsl(d) < tiny) d = tiny;
        c = b + an / c;
        if (fabsl(c) < tiny) c = tiny;
        d = 1 / d;
        ld del = d * c;
        h *= del;
        if (fabsl(del - 1) <= 2 * LDBL_EPSILON) break;
    }
    return y * h;        /* Gamma(a,y) e^y y^{-a} = h, times y */
}

/* log Gamma(a, y) for y >= 0 */
static ld log_upper_gamma(ld a, ld y)
{
    if (y == 0) return lgammal(a);
    if (y < a + 1) {
        ld g = expl(a * logl(y) - y - lgammal(a)) * lower_series(a, y);   /* gamma(a, y) / Gamma(a) */
        return lgammal(a) + log1pl(-g);
    }
    return -y + (a - 1) * logl(y) + logl(upper_cf(a, y));
}

/* log gamma(a, y) for y > 0 (no cancellation below a + 1) */
static ld log_lower_gamma(ld a, ld y)
{
    if (y < a + 1) return a * logl(y) - y + logl(lower_series(a, y));
    ld q = expl(-y + (a - 1) * logl(y) - lgammal(a)) * upper_cf(a, y);    /* Gamma(a, y) / Gamma(a) */
    return lgammal(a) + log1pl(-q);
}


/* ---- one side of the density ---- */

typedef struct {
    ld alpha, beta;   /* beta of this side (the left side mirrors it) */
    ld nu, a;         /* lambda - 1/2, lambda + 1/2 */
    ld r;             /* base rate alpha - beta */
    ld logA;
    ld h;             /* trapezoid step in s */
    ld lp;            /* log of this side's mass */
} rside;

/*
 * log of A int_0^inf cosh(nu s) c(s)^{-a} G(a, c(s) x) ds by the trapezoidal
 * rule, G the upper (upper = 1) or lower incomplete gamma function.
 *
 * Each term is formed from logarithms of moderate size only, because an
 * absolute rounding e in a term's logarithm is a relative error e in the
 * term, and the plain logs (nu s, a log c, a log x) reach thousands.  With
 * a - nu = 1,
 *     cosh(nu s) c^{-a} = R(s) (2/alpha)^nu / c,
 *     log R(s) = log1p(e^{-2 nu s}) - log 2 - nu log1p(e^{-2s} - (2 beta/alpha) e^{-s})
 * (R tends to 1/2 as s grows); the lower terms are
 *     R (2/alpha)^nu x gamma(a, y)/y,   y = c x,
 * with log x summed outside; the upper terms, times e^{r x}, are
 *     R (2/alpha)^nu Gamma(a, y) e^{r x} / c,
 * and when every y is past a + 1 (r x >= a + 1) Gamma(a, y) e^{r x} =
 * e^{-(c - r) x} y^{a-1} CF with c - r = 2 alpha sinh^2(s/2) and (a - 1) log x
 * summed outside.  The terms are summed relative to the largest so far (the
 * lower ones first grow while y << 1); the sum stops after 8 terms in a row
 * below 1e-23 of it, once past the largest.
 */
static ld log_trapezoid(const rside* S, ld x, int upper)
{
    /* step: d/10 for the strip, and 0.5/sqrt(alpha x) so that the growth of
       e^{-c x} off the axis, e^{alpha (1 - cos t) x} at height t, stays
       below the trapezoid's e^{-2 pi t / h} (their balance point leaves
       e^{-2 pi^2 / (h^2 alpha x)} < e^{-78}) */
    const ld h = fminl(S->h, 0.5L / sqrtl(S->alpha * x));
    const ld a = S->a, nu = S->nu, ba = S->beta / S->alpha;
    const int far = upper && S->r * x >= a + 1;
    const ld lx = x > 0 ? logl(x) : 0;
    ld sum = 0, shift = -INFINITY, prev = -INFINITY;
    int small = 0, falling = 0;
    for (long k = 0; k < 20000000L; ++k) {
        const ld s = k * h;
        const ld es = expl(-s);
        const ld c = S->alpha * coshl(s) - S->beta;
        if (!isfinite(c)) break;
        const ld logR = log1pl(expl(-2 * nu * s)) - LN2L - nu * log1pl(es * es - 2 * ba * es);
        const ld y = c * x;
        ld lg;
        if (!upper) {
            /* log(gamma(a, y)/y) */
            lg = y < a + 1 ? (a - 1) * logl(y) - y + logl(lower_series(a, y)) : log_lower_gamma(a, y) - logl(y);
        } else if (far) {
            /* log(Gamma(a, y) e^{r x} / c) less (a - 1) log x */
            const ld sh = sinhl(s / 2);
            lg = -2 * S->alpha * sh * sh * x + (a - 2) * logl(c) + logl(upper_cf(a, y));
        } else {
            lg = log_upper_gamma(a, y) + S->r * x - logl(c);
        }
        const ld lt = logR + lg + (k == 0 ? -LN2L : 0);
        if (lt > shift) {
            sum = sum * expl(shift - lt) + 1;
            shift = lt;
        } else {
            sum += expl(lt - shift);
        }
        if (lt < prev) falling = 1;
        prev = lt;
        if (falling && k > 8 && lt - shift < logl(1e-23L * sum)) {
            if (++small >= 8) break;
        } else {
            small = 0;
        }
    }
    const ld outside = nu * logl(2 / S->alpha) + (!upper ? lx : far ? (a - 1) * lx : 0);
    return S->logA + logl(h) + outside + shift + logl(sum) - (upper ? S->r * x : 0);
}

/* log T(x) = log int_x^inf f, x >= 0 */
static ld log_tail(const rside* S, ld x) { return log_trapezoid(S, x, 1); }

/* M(x) = int_0^x f, x >= 0 */
static ld central_mass(const rside* S, ld x) { return x > 0 ? expl(log_trapezoid(S, x, 0)) : 0; }

static void side_init(rside* S, ld lambda, ld alpha, ld beta)
{
    S->alpha = alpha;
    S->beta = beta;
    S->nu = lambda - 0.5L;
    S->a = lambda + 0.5L;
    S->r = alpha - beta;
    S->logA = lambda * logl((alpha - beta) * (alpha + beta)) - S->nu * logl(2 * alpha) - 0.5L * logl(PIL) -
              lgammal(lambda);
    /* the s-integrand is analytic where c(s) != 0, |Im s| < arccos(beta/alpha),
       and decays (Re c > 0 far out) only for |Im s| < pi/2 */
    ld d = fminl(acosl(beta / alpha), PIL / 2);
    S->h = d / 10;
    S->lp = log_tail(S, 0);
}

static uint64_t dbits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }
static double bitsd(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }

/* X >= 0 with the upper tail beyond X equal to p+ e^{-r v}, v >= 0 */
static double solve(const rside* S, ld v)
{
    ld rv = S->r * v;
    int central = rv <= LN2L;
    ld target = central ? -expl(S->lp) * expm1l(-rv) : S->lp - rv;
#define RES(xv) (central ? (central_mass(S, (ld)(xv)) - target) : (target - log_tail(S, (ld)(xv))))
    if (v == 0) return 0.0;
    /* bracket by bits: the map is monotone and within a few e-folds of
       x = v far out, so start the search from [v/64, 64 v + 64] clipped to
       the double range, widening if the residual says so */
    uint64_t lo = 0, hi = dbits(DBL_MAX);
    double xl = (double)(v / 64), xh = (double)(64 * v + 64);
    if (isfinite(xh) && RES(xh) >= 0) hi = dbits(xh);
    if (xl > 0 && RES(xl) < 0) lo = dbits(xl);
    if (hi == dbits(DBL_MAX) && RES(DBL_MAX) < 0) return INFINITY;
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (RES(bitsd(mid)) < 0) lo = mid; else hi = mid;
    }
    double a = bitsd(lo), b = bitsd(hi);
    ld ra = fabsl(RES(a)), rb = fabsl(RES(b));
#undef RES
    return ra < rb ? a : b;
}

typedef struct { rside right, left; int ok; } rctx;

static int params_ok(double lambda, double alpha, double beta)
{
    return isfinite(lambda) && isfinite(alpha) && isfinite(beta) && lambda >= 1 && lambda <= 64 && alpha > fabs(beta);
}

static void rctx_init(rctx* c, double lambda, double alpha, double beta)
{
    c->ok = params_ok(lambda, alpha, beta);
    if (!c->ok) return;
    side_init(&c->right, lambda, alpha, beta);
    side_init(&c->left, lambda, alpha, -(ld)beta);
}

static double map_one(const rctx* c, double v)
{
    if (!c->ok || isnan(v)) return NAN;
    if (isinf(v)) return v;
    if (v >= 0) return solve(&c->right, v);
    return -solve(&c->left, -(ld)v);
}

typedef struct {
    const rctx* c;
    const double* v;
    double* out;
    size_t lo, hi;
} job;

static void* worker(void* p)
{
    job* j = (job*)p;
    for (size_t i = j->lo; i < j->hi; ++i) j->out[i] = map_one(j->c, j->v[i]);
    return NULL;
}

int oracle_vgr_map(const double* v, double* out, size_t n, double lambda, double alpha, double beta, int threads)
{
    rctx c;
    rctx_init(&c, lambda, alpha, beta);
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    if ((size_t)threads > n) threads = n ? (int)n : 1;
    pthread_t t[64];
    job jobs[64];
    size_t per = (n + threads - 1) / threads;
    for (int i = 0; i < threads; ++i) {
        jobs[i].c = &c;
        jobs[i].v = v;
        jobs[i].out = out;
        jobs[i].lo = i * per < n ? i * per : n;
        jobs[i].hi = (i + 1) * per < n ? (i + 1) * per : n;
        pthread_create(&t[i], NULL, worker, &jobs[i]);
    }
    for (int i = 0; i < threads; ++i) pthread_join(t[i], NULL);
    return c.ok ? 0 : -1;
}

/* log p+ and log p- of the target */
int oracle_vgr_masses(double lambda, double alpha, double beta, double* lp, double* lm)
{
    rctx c;
    rctx_init(&c, lambda, alpha, beta);
    if (!c.ok) return -1;
    *lp = (double)c.right.lp;
    *lm = (double)c.left.lp;
    return 0;
}

/* log(1 - F(x)) for x >= 0, log F(x) for x < 0 */
double oracle_vgr_log_tail(double x, double lambda, double alpha, double beta)
{
    rctx c;
    rctx_init(&c, lambda, alpha, beta);
    if (!c.ok || isnan(x)) return NAN;
    return x >= 0 ? (double)log_tail(&c.right, x) : (double)log_tail(&c.left, -(ld)x);
}

/* int_0^|x| f on the side of x (for pins of the central form) */
double oracle_vgr_central_mass(double x, double lambda, double alpha, double beta)
{
    rctx c;
    rctx_init(&c, lambda, alpha, beta);
    if (!c.ok || isnan(x)) return NAN;
    return x >= 0 ? (double)central_mass(&c.right, x) : (double)central_mass(&c.left, -(ld)x);
}

/* the incomplete gamma pieces, exposed for pins: log Gamma(a, y), log gamma(a, y) */
double oracle_vgr_log_upper_gamma(double a, double y) { return (double)log_upper_gamma(a, y); }
double oracle_vgr_log_lower_gamma(double a, double y) { return (double)log_lower_gamma(a, y); }

/*
 * hyperbolic.c -- oracle for the exponential -> hyperbolic recycling map.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product library
 * calls, links or loads this file, and it shares no code with it.
 *
 * What is computed (Shaw, Luu & Brickman, "Quantile Mechanics II", Section
 * 8.1).  Target: the hyperbolic density with mu = 0,
 *     f(x) = C exp(-alpha sqrt(delta^2 + x^2) + beta x),  |beta| < alpha, delta > 0,
 * C its normalising constant.  Base: the two-sided exponential density
 *     f0(v) = p+ (alpha - beta) e^{-(alpha-beta) v}   (v > 0),
 *             p- (alpha + beta) e^{(alpha+beta) v}    (v < 0),
 * with p+ and p- the target's masses on x > 0 and x < 0, so that the map
 * keeps Q(0) = 0.  The map is Q(v) = F^{-1}(F0(v)):
 *     v >= 0:  1 - F(Q) = p+ e^{-(alpha-beta) v},
 *     v <  0:  F(Q)     = p- e^{(alpha+beta) v}.
 * v < 0 is the mirror image: x -> -x and beta -> -beta exchange the two
 * sides, so Q(v; beta) = -Q(-v; -beta) is used for it.
 *
 * Method.  With x = delta sinh s (so sqrt(delta^2 + x^2) = delta cosh s),
 * f(x) dx = C delta e^{-delta gamma} e^{E(s)} cosh s ds, where
 *     E(s) = -alpha delta cosh s + beta delta sinh s + delta gamma <= 0,
 * gamma = sqrt(alpha^2 - beta^2), with its maximum 0 at tanh s = beta/alpha:
 * a smooth integrand that decays double-exponentially, integrated by
 * adaptive Gauss-Legendre (20 nodes per panel, panels halved until two
 * halves agree with the whole) in x87 extended precision.  The constant C
 * is not taken from its closed form: the density is normalised by the same
 * quadrature (the closed form with K1 is a pin in the tests).  Upper tails
 * are carried as logarithms (the integral past a point beyond the peak is
 * scaled by e^{E} at that point), so they stay accurate far below the
 * smallest double.  The defining equation is solved by bisection over the
 * IEEE-754 bit pattern of x >= 0, ending on two adjacent doubles, the one
 * with the smaller residual returned -- with the equation in its central
 * form int_0^x f = p+ (1 - e^{-(alpha-beta) v}) (formed with expm1) while
 * (alpha - beta) v <= log 2, in its tail form in logarithms beyond.
 *
 * Error behaviour: per element; NaN in -> NaN out, v = +-inf -> +-inf,
 * invalid parameters (alpha <= |beta|, delta <= 0, non-finite) -> NaN.
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <unistd.h>

typedef long double ld;

#define GL_N 20
static ld gl_x[GL_N], gl_w[GL_N];
static pthread_once_t gl_once = PTHREAD_ONCE_INIT;

/* Gauss-Legendre nodes and weights on [-1, 1]: Newton on P_N from the
   Chebyshev-like first guesses, P_N by its three-term recurrence. */
static void gl_init(void)
{
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < GL_N; ++i) {
        ld x = cosl(pi * (i + 0.75L) / (GL_N + 0.5L)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1, p1 = x;
            for (int k = 2; k <= GL_N; ++k) {
                ld p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = GL_N * (x * p1 - p0) / (x * x - 1);
            ld dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-30L) break;
        }
        gl_x[i] = x;
        gl_w[i] = 2 / ((1 - x * x) * dp * dp);
    }
}

typedef struct {
    ld ad, bd, dg;   /* alpha delta, beta delta, delta gamma */
    ld speak;        /* the peak of E: tanh s = beta/alpha */
    ld ks;           /* log of the constant that turns the s-integral into mass: -log N */
    ld lp_plus;      /* log p+ */
    ld rate;         /* alpha - beta */
    ld delta;
} hside;

/* E(s) = -alpha delta cosh s + beta delta sinh s + delta gamma, formed as
   -2 delta gamma sinh^2((s - s_peak)/2) (alpha = gamma cosh s_peak,
   beta = gamma sinh s_peak): the same number without the cancellation of
   the first form when beta is close to alpha */
static ld E_of(const hside* h, ld s)
{
    ld q = sinhl(0.5L * (s - h->speak));
    return -2 * h->dg * q * q;
}

/* E(a + u) - E(a) = -2 sinh(u/2) (alpha delta sinh(a + u/2) - beta delta cosh(a + u/2))
   = -2 delta gamma sinh(u/2) sinh(a + u/2 - s_peak), exact in u however large
   a is (a + u itself may round to a) */
static ld dE(const hside* h, ld a, ld u)
{
    ld m = a + 0.5L * u;
    return -2 * sinhl(0.5L * u) * h->dg * sinhl(m - h->speak);   /* alpha sinh m - beta cosh m = gamma sinh(m - s_peak) */
}

/* The integrand at s = a + u: e^{E(s) - shift} cosh s, with E(a) - shift
   given as ea (so that it is 0 where shift = E(a)) */
static ld integrand(const hside* h, ld a, ld ea, ld u) { return expl(ea + dE(h, a, u)) * coshl(a + u); }

static ld gl_panel(const hside* h, ld a, ld ea, ld u0, ld u1)
{
    ld c = 0.5L * (u0 + u1), r = 0.5L * (u1 - u0), sum = 0;
    for (int i = 0; i < GL_N; ++i) sum += gl_w[i] * integrand(h, a, ea, c + r * gl_x[i]);
    return sum * r;
}

/* Halve a panel until its two halves agree with it to tol, or to the
   rounding of the integrand itself: E carries an absolute error of a few
   ulps of |E|, a relative error of e^E, so no estimate is better than about
   |E| eps (the integrand is positive: the sums do not cancel). */
static ld gl_adapt(const hside* h, ld a, ld ea, ld u0, ld u1, ld whole, ld tol, int depth)
{
    ld m = 0.5L * (u0 + u1);
    ld left = gl_panel(h, a, ea, u0, m), right = gl_panel(h, a, ea, m, u1);
    ld diff = fabsl(left + right - whole);
    ld noise = 64 * LDBL_EPSILON * (1 + fabsl(E_of(h, a + u0)) + fabsl(E_of(h, a + u1)));
    if (depth >= 30 || diff <= tol || diff <= noise * (left + right)) return left + right;
    return gl_adapt(h, a, ea, u0, m, left, 0.5L * tol, depth + 1) +
           gl_adapt(h, a, ea, m, u1, right, 0.5L * tol, depth + 1);
}

/* int over s in [a + u0, a + u1] of e^{E(s) - shift} cosh s ds (ea = E(a) -
   shift), to 1e-21 relative, or to the absolute tolerance floor when that is
   larger (a panel that is a negligible part of a larger sum) */
static ld integrate_tol(const hside* h, ld a, ld ea, ld u0, ld u1, ld floor_tol)
{
    if (!(u1 > u0)) return 0;
    ld whole = gl_panel(h, a, ea, u0, u1);
    ld tol = 1e-21L * fabsl(whole);
    if (tol < floor_tol) tol = floor_tol;
    return gl_adapt(h, a, ea, u0, u1, whole, tol + 1e-4000L, 0);
}

/* int_a^b e^{E(s) - shift} cosh s ds */
static ld integrate(const hside* h, ld a, ld b, ld shift) { return integrate_tol(h, a, E_of(h, a) - shift, 0, b - a, 0); }

/* int_a^inf e^{E(s) - shift} cosh s ds, by panels until they vanish.  Past
   the peak the integrand falls like e^{E'(a)(s - a)} at first (and faster
   after), so the panels are 1/|E'(a)| wide, at most 1: each holds a fixed
   share of the decay, however far out a lies.  The panels are placed by
   their offset from a, which resolves widths far below the spacing of
   numbers near a. */
static ld integrate_to_inf(const hside* h, ld a, ld shift)
{
    ld slope = h->dg * sinhl(a - h->speak);     /* -E'(a) */
    ld w = (a > h->speak && slope > 1) ? 1 / slope : 1;
    ld ea = E_of(h, a) - shift, sum = 0;
    for (int k = 0; k < 100000; ++k) {
        ld p = integrate_tol(h, a, ea, k * w, (k + 1) * w, 1e-22L * sum);
        sum += p;
        if (a + k * w > h->speak && p <= 1e-30L * sum) break;
    }
    return sum;
}

/* log of the upper-tail mass 1 - F(x), x >= 0 */
static ld log_upper(const hside* h, ld x)
{
    ld S = asinhl(x / h->delta);
    if (S > h->speak) {
        ld e = E_of(h, S);
        return h->ks + e + logl(integrate_to_inf(h, S, e));   /* e - shift is exactly 0 */
    }
    return h->ks + logl(integrate(h, S, h->speak, 0) + integrate_to_inf(h, h->speak, 0));
}

/* mass of [0, x], x >= 0: directly while x is within two units of s past
   the peak (the range the equation's central form is used on), else as
   p+ minus the upper tail (there only its sign matters to the bisection,
   and an integral over a huge range of s is not worth forming) */
static ld central_mass(const hside* h, ld x)
{
    ld S = asinhl(x / h->delta);
    if (S <= (h->speak > 0 ? h->speak : 0) + 2) return expl(h->ks) * integrate(h, 0, S, 0);
    return expl(h->lp_plus) - expl(log_upper(h, x));
}

static void hside_init(hside* h, ld alpha, ld beta, ld delta)
{
    pthread_once(&gl_once, gl_init);
    ld gamma = sqrtl((alpha - beta) * (alpha + beta));
    h->ad = alpha * delta;
    h->bd = beta * delta;
    h->dg = delta * gamma;
    h->speak = atanhl(beta / alpha);
    h->delta = delta;
    h->rate = alpha - beta;
    h->ks = 0;
    ld total = integrate(h, h->speak - 1, h->speak + 1, 0) + integrate_to_inf(h, h->speak + 1, 0);
    /* the left side: s -> -s with beta -> -beta */
    hside m = *h;
    m.bd = -h->bd;
    m.speak = -h->speak;
    total += integrate_to_inf(&m, 1 - h->speak, 0);
    h->ks = -logl(total);
    h->lp_plus = log_upper(h, 0);
}

static uint64_t dbits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }
static double bitsd(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }

/* X >= 0 with the upper tail beyond X equal to p+ e^{-rate v}, v >= 0 */
static double solve_side(const hside* h, ld v)
{
    ld a = h->rate * v;
    int central = a <= 0.69314718055994530942L;
    ld target = central ? -expl(h->lp_plus) * expm1l(-a) : h->lp_plus - a;
    /* residual oriented to increase with x */
    #define RES(xv) (central ? (central_mass(h, (ld)(xv)) - target) : (target - log_upper(h, (ld)(xv))))
    uint64_t lo = 0, hi = dbits(DBL_MAX);
    if (RES(DBL_MAX) < 0) return INFINITY;
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (RES(bitsd(mid)) < 0) lo = mid; else hi = mid;
    }
    double xl = bitsd(lo), xh = bitsd(hi);
    ld rl = fabsl(RES(xl)), rh = fabsl(RES(xh));
    #undef RES
    return rl < rh ? xl : xh;
}

typedef struct { hside right, left; int ok; } hctx;

static void hctx_init(hctx* c, double alpha, double beta, double delta)
{
    c->ok = isfinite(alpha) && isfinite(beta) && isfinite(delta) && delta > 0 && alpha > fabs(beta);
    if (!c->ok) return;
    hside_init(&c->right, alpha, beta, delta);
    hside_init(&c->left, alpha, -beta, delta);
}

static double hyp_map1(const hctx* c, double v)
{
    if (!c->ok || isnan(v)) return NAN;
    if (v == 0) return v;
    if (isinf(v)) return v;
    if (v > 0) return solve_side(&c->right, v);
    return -solve_side(&c->left, -(ld)v);
}

double oracle_hyperbolic_map1(double v, double alpha, double beta, double delta)
{
    hctx c;
    hctx_init(&c, alpha, beta, delta);
    return hyp_map1(&c, v);
}

/* log p+ and log p- (the target's masses on each side), and log C */
int oracle_hyperbolic_masses(double alpha, double beta, double delta, double* lp_plus, double* lp_minus,
                             double* log_c)
{
    hctx c;
    hctx_init(&c, alpha, beta, delta);
    if (!c.ok) return -1;
    *lp_plus = (double)c.right.lp_plus;
    *lp_minus = (double)c.left.lp_plus;
    /* f dx = e^{ks} e^{E} cosh s ds and f dx = C delta e^{-delta gamma} e^{E} cosh s ds */
    *log_c = (double)(c.right.ks + c.right.dg - logl(c.right.delta));
    return 0;
}

/* log of the upper tail 1 - F(x) for x >= 0, and of F(x) for x < 0 */
double oracle_hyperbolic_log_tail(double x, double alpha, double beta, double delta)
{
    hctx c;
    hctx_init(&c, alpha, beta, delta);
    if (!c.ok || isnan(x)) return NAN;
    return x >= 0 ? (double)log_upper(&c.right, x) : (double)log_upper(&c.left, -(ld)x);
}

typedef struct {
    const hctx* c;
    const double* in;
    double* out;
    size_t begin, end;
} hjob;

static void* hrun(void* p)
{
    hjob* j = (hjob*)p;
    for (size_t i = j->begin; i < j->end; ++i) j->out[i] = hyp_map1(j->c, j->in[i]);
    return NULL;
}

int oracle_hyperbolic_map(const double* v, double* x, size_t n, double alpha, double beta, double delta,
                          int nthreads)
{
    hctx c;
    hctx_init(&c, alpha, beta, delta);
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if ((size_t)nthreads > n) nthreads = n > 0 ? (int)n : 1;
    pthread_t th[64];
    hjob jobs[64];
    size_t per = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].c = &c;
        jobs[t].in = v;
        jobs[t].out = x;
        jobs[t].begin = t * per < n ? t * per : n;
        jobs[t].end = (t + 1) * per < n ? (t + 1) * per : n;
        pthread_create(&th[t], NULL, hrun, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

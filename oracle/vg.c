/*
 * vg.c -- oracle for the exponential -> variance-gamma recycling map with
 * integer lambda.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product library
 * calls, links or loads this file, and it shares no code with it.
 *
 * What is computed (Shaw, Luu & Brickman, "Quantile Mechanics II", Section
 * 8.2).  Target: the variance-gamma density (mu = 0)
 *     f(x) = (alpha^2 - beta^2)^lambda e^{beta x} |x|^{lambda - 1/2} K_{lambda-1/2}(alpha |x|)
 *            / ((2 alpha)^{lambda - 1/2} sqrt(pi) Gamma(lambda)),
 * lambda > 0, |beta| < alpha.  For lambda = n + 1 (n = 0, 1, 2, ...) the
 * Bessel function is elementary (DLMF 10.49.12):
 *     K_{n+1/2}(z) = sqrt(pi/(2z)) e^{-z} sum_{k=0}^{n} (n+k)! / (k! (n-k)!) (2z)^{-k},
 * so on x > 0
 *     f(x) = A e^{-r x} sum_{k=0}^{n} c_k x^{n-k},   r = alpha - beta,
 *     c_k = (n+k)! / (k! (n-k)! (2 alpha)^k),
 *     A = (alpha^2 - beta^2)^lambda sqrt(pi/(2 alpha)) / ((2 alpha)^{lambda-1/2} sqrt(pi) n!),
 * and with int_x^inf t^m e^{-r t} dt = m! e^{-r x} sum_{j<=m} (r x)^j / j! / r^{m+1}
 * every mass is a finite sum.  Base and map as for the hyperbolic target
 * (Section 8.1, the same two-sided exponential base with the target's
 * masses p+, p-): 1 - F(Q) = p+ e^{-r v} for v >= 0, and the mirror image
 * (beta -> -beta) for v < 0.
 *
 * Method: the equation is solved by bisection over the IEEE-754 bit
 * pattern of x >= 0, ending on two adjacent doubles, the one with the
 * smaller residual returned; in its central form
 * M(x) = int_0^x f = p+ (1 - e^{-r v}) (M by the series of the lower
 * incomplete gamma function, which has no cancellation) while r v <= ln 2,
 * in logarithms of the tail beyond.  Long double throughout.
 *
 * Error behaviour: per element; NaN -> NaN, +-inf -> +-inf; parameters
 * outside integer lambda in [1, 64], alpha > |beta|, all finite -> NaN.
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <unistd.h>

typedef long double ld;

#define VG_NMAX 63

typedef struct {
    int n;            /* lambda - 1 */
    ld r;             /* rate of the side */
    ld logA;          /* log A */
    ld c[VG_NMAX + 1];
    ld lp;            /* log of this side's mass */
} vside;

/* log of int_x^inf t^m e^{-r t} dt = log m! - r x + log sum_{j<=m} (r x)^j / j! - (m+1) log r;
   for y = r x > m the sum is taken relative to its last term y^m/m!, so
   that it cannot overflow however large x is */
static ld log_upper_gamma(int m, ld r, ld x)
{
    ld y = r * x;
    ld lsum;
    if (y > m && m > 0) {
        ld term = 1, sum = 1;
        for (int j = m; j >= 1; --j) {
            term *= j / y;
            sum += term;
        }
        lsum = m * logl(y) - lgammal((ld)m + 1) + logl(sum);
    } else {
        ld term = 1, sum = 1;
        for (int j = 1; j <= m; ++j) {
            term *= y / j;
            sum += term;
        }
        lsum = logl(sum);
    }
    return lgammal((ld)m + 1) - y + lsum - (m + 1) * logl(r);
}

/* int_0^x t^m e^{-r t} dt = m! / r^{m+1} e^{-y} sum_{j>m} y^j / j!, y = r x
   (no cancellation); far out, where that series is long and e^{-y} may
   underflow, the whole integral m!/r^{m+1} less the (then tiny) upper part */
static ld lower_gamma(int m, ld r, ld x)
{
    ld y = r * x;
    if (y > m + 60) return expl(lgammal((ld)m + 1) - (m + 1) * logl(r)) - expl(log_upper_gamma(m, r, x));
    ld term = expl(-y), sum = 0;
    for (int j = 1; j <= m; ++j) term *= y / j;   /* e^{-y} y^m / m! */
    for (int j = m + 1; j < 100000; ++j) {
        term *= y / j;
        sum += term;
        if (term <= 1e-22L * sum) break;
    }
    return expl(lgammal((ld)m + 1) - (m + 1) * logl(r)) * sum;
}

/* log(1 - F(x)) on this side, x >= 0: log A + log sum_k c_k int_x^inf t^{n-k} e^{-r t} dt
   (positive terms, summed in the scale of the largest) */
static ld log_tail(const vside* s, ld x)
{
    ld l[VG_NMAX + 1], mx = -INFINITY;
    for (int k = 0; k <= s->n; ++k) {
        l[k] = logl(s->c[k]) + log_upper_gamma(s->n - k, s->r, x);
        if (l[k] > mx) mx = l[k];
    }
    ld sum = 0;
    for (int k = 0; k <= s->n; ++k) sum += expl(l[k] - mx);
    return s->logA + mx + logl(sum);
}

static ld central_mass(const vside* s, ld x)
{
    ld sum = 0;
    for (int k = 0; k <= s->n; ++k) sum += s->c[k] * lower_gamma(s->n - k, s->r, x);
    return expl(s->logA) * sum;
}

static void side_init(vside* s, int n, ld alpha, ld beta)
{
    s->n = n;
    s->r = alpha - beta;
    ld lam = n + 1;
    s->logA = lam * logl((alpha - beta) * (alpha + beta)) + 0.5L * logl(3.141592653589793238462643383279502884L / (2 * alpha)) -
              (lam - 0.5L) * logl(2 * alpha) - 0.5L * logl(3.141592653589793238462643383279502884L) - lgammal(lam);
    for (int k = 0; k <= n; ++k)
        s->c[k] = expl(lgammal((ld)(n + k) + 1) - lgammal((ld)k + 1) - lgammal((ld)(n - k) + 1) - k * logl(2 * alpha));
    s->lp = log_tail(s, 0);
}

static uint64_t dbits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }
static double bitsd(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }

/* X >= 0 with the upper tail beyond X equal to p e^{-r v}, v >= 0 */
static double solve(const vside* s, ld v)
{
    ld a = s->r * v;
    int central = a <= 0.69314718055994530942L;
    ld target = central ? -expl(s->lp) * expm1l(-a) : s->lp - a;
#define RES(xv) (central ? (central_mass(s, (ld)(xv)) - target) : (target - log_tail(s, (ld)(xv))))
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

typedef struct { vside right, left; int ok; } vctx;

static int params_ok(double lambda, double alpha, double beta)
{
    return isfinite(lambda) && isfinite(alpha) && isfinite(beta) && lambda >= 1 && lambda <= VG_NMAX + 1 &&
           lambda == floor(lambda) && alpha > fabs(beta);
}

static void vctx_init(vctx* c, double lambda, double alpha, double beta)
{
    c->ok = params_ok(lambda, alpha, beta);
    if (!c->ok) return;
    side_init(&c->right, (int)lambda - 1, alpha, beta);
    side_init(&c->left, (int)lambda - 1, alpha, -(ld)beta);
}

static double map_one(const vctx* c, double v)
{
    if (!c->ok || isnan(v)) return NAN;
    if (isinf(v)) return v;
    if (v >= 0) return solve(&c->right, v);
    return -solve(&c->left, -(ld)v);
}

typedef struct {
    const vctx* c;
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

int oracle_vg_map(const double* v, double* out, size_t n, double lambda, double alpha, double beta, int threads)
{
    vctx c;
    vctx_init(&c, lambda, alpha, beta);
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
int oracle_vg_masses(double lambda, double alpha, double beta, double* lp, double* lm)
{
    vctx c;
    vctx_init(&c, lambda, alpha, beta);
    if (!c.ok) return -1;
    *lp = (double)c.right.lp;
    *lm = (double)c.left.lp;
    return 0;
}

/* log(1 - F(x)) for x >= 0, log F(x) for x < 0 */
double oracle_vg_log_tail(double x, double lambda, double alpha, double beta)
{
    vctx c;
    vctx_init(&c, lambda, alpha, beta);
    if (!c.ok || isnan(x)) return NAN;
    return x >= 0 ? (double)log_tail(&c.right, x) : (double)log_tail(&c.left, -(ld)x);
}

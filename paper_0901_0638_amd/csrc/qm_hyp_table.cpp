/*
 * qm_hyp_table.cpp -- host builder of the tables of the two-sided
 * exponential base: exponential -> hyperbolic (Section 8.1, from the
 * recycling ODE, below) and exponential -> variance-gamma for real lambda in
 * [1, 8] (Section 8.2: integer lambda solved directly from closed-form
 * masses, VGSide; other lambda from the recycling ODE, VGRealSide).
 * Both fit the same cells through one interface (SideMap), so both run in
 * the same kernel.
 *
 * Section 8.1: the hyperbolic target (mu = 0)
 *     f(x) = C exp(-alpha sqrt(delta^2 + x^2) + beta x),
 *     C = gamma / (2 alpha delta K_1(delta gamma)),  gamma = sqrt(alpha^2 - beta^2),
 * is reached from the two-sided exponential base with the target's masses
 * p+ and p- on each side and rates alpha - beta (right), alpha + beta
 * (left), so that Q(0) = 0.  With H(x) = alpha x / sqrt(delta^2 + x^2) - beta
 * (minus the log-derivative of f), the right map solves the recycling ODE
 *     Q'' + (alpha - beta) Q' = H(Q) Q'^2,  Q(0) = 0,
 *     Q'(0) = p+ (alpha - beta) / f(0) = 2 p+ (alpha - beta) (alpha delta / gamma) K_1(delta gamma) e^{alpha delta},
 * and the left map is the right map of the mirrored target (beta -> -beta),
 * reflected: Q(v) = -Q~(-v).
 *
 * As for the Student t builder, the ODE is integrated by the Taylor-series
 * method in __float128 -- here the series of H(Q) comes from those of
 * Q^2 + delta^2 and of its inverse square root (J. C. P. Miller's
 * recurrence for a power of a series) -- and from both ends: outwards from
 * the centre conditions, and inwards from an anchor v_a, where Q solves the
 * tail condition log(1 - F(Q)) = log p+ - (alpha - beta) v_a directly;
 * outward integration would amplify any error by e^{(alpha-beta) v}.
 * Beyond v_a, Q is that direct solution (Newton), with the tail mass in
 * closed form up to one smooth integral: with s = asinh(x/delta) and
 * c = cosh(s - s_peak) (alpha = gamma cosh s_peak, beta = gamma sinh s_peak),
 *     1 - F(x) = (C delta / z) e^{-z c0} (e^{s_peak} + cosh(s_peak) K),
 *     K = int_0^inf e^{-t} (h(c0 + t/z) - 1) dt,  h(c) = c / sqrt(c^2 - 1),
 * z = delta gamma, c0 = c at x, z c0 = alpha sqrt(delta^2 + x^2) - beta x;
 * K by Gauss-Laguerre quadrature, accurate once D = z (c0 - 1) is large
 * (the singularity of h at c = 1 lies a distance D to the left of t = 0).
 * An explicit integrator cannot take steps much longer than 1/(alpha - beta)
 * there (the decaying mode of the backward direction limits them), which
 * would make the far range, out to where the large-v form below holds,
 * cost millions of steps.  The table holds R(v) = Q(v)/v in
 * cells of t = 1 + v / v0, eight per octave of t: uniform cells on
 * [0, v0), then cells whose relative width tends to 1/8 (Q is nearly
 * v + const far out, and curved on the scale delta near 0).  Both sides
 * share v0, a power of 2.
 * Each cell holds the degree-11 Chebyshev interpolant of R as monomials in
 * d = v - centre, checked against the solution.  Beyond the last
 * octave, Q = v + c0 + c1/v + c2/v^2 (the expansion of the tail condition
 * for large v, derived at solve_side), checked there too.
 */
#include <quadmath.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "qm_hyp_table.h"

namespace qm {
namespace {

typedef __float128 fq;

constexpr int TM = 32;              /* Taylor order of the integrator */
constexpr int GLN = 24;             /* Gauss-Legendre nodes per panel */

struct GL {
    fq x[GLN], w[GLN];
    GL()
    {
        for (int i = 0; i < GLN; ++i) {
            fq x0 = cosq(M_PIq * (i + 0.75Q) / (GLN + 0.5Q)), dp = 0;
            for (int it = 0; it < 100; ++it) {
                fq p0 = 1, p1 = x0;
                for (int k = 2; k <= GLN; ++k) {
                    fq p2 = ((2 * k - 1) * x0 * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = GLN * (x0 * p1 - p0) / (x0 * x0 - 1);
                fq dx = p1 / dp;
                x0 -= dx;
                if (fabsq(dx) < 1e-33Q) break;
            }
            x[i] = x0;
            w[i] = 2 / ((1 - x0 * x0) * dp * dp);
        }
    }
};

const GL& gl()
{
    static const GL g;
    return g;
}

/* One side of the target: parameters and its tail masses. */
struct Side {
    fq alpha, beta, delta, gamma, rate;
    fq ad, bd, dg, speak;   /* alpha delta, beta delta, delta gamma, peak of E in s */
    fq log_c;               /* log C */
    fq log_p;               /* log of this side's mass */

    /* E(s) = -alpha delta cosh s + beta delta sinh s + delta gamma
            = -delta gamma (cosh(s - s_peak) - 1) = -2 delta gamma sinh^2((s - s_peak)/2) <= 0
       (alpha = gamma cosh s_peak, beta = gamma sinh s_peak): no cancellation,
       however close beta is to alpha */
    fq E(fq s) const
    {
        fq h = sinhq((s - speak) / 2);
        return -2 * dg * h * h;
    }

    fq panel(fq a, fq b, fq shift) const
    {
        const GL& g = gl();
        fq c = (a + b) / 2, r = (b - a) / 2, sum = 0;
        for (int i = 0; i < GLN; ++i) {
            fq s = c + r * g.x[i];
            sum += g.w[i] * expq(E(s) - shift) * coshq(s);
        }
        return sum * r;
    }

    fq adapt(fq a, fq b, fq shift, fq whole, fq tol, int depth) const
    {
        fq m = (a + b) / 2;
        fq l = panel(a, m, shift), r = panel(m, b, shift);
        fq diff = fabsq(l + r - whole);
        fq noise = 1e-32Q * (1 + fabsq(E(a)) + fabsq(E(b)));
        if (depth >= 30 || diff <= tol || diff <= noise * (l + r)) return l + r;
        return adapt(a, m, shift, l, tol / 2, depth + 1) + adapt(m, b, shift, r, tol / 2, depth + 1);
    }

    /* int_a^b e^{E(s) - shift} cosh s ds */
    fq integral(fq a, fq b, fq shift, fq floor_tol = 0) const
    {
        if (!(b > a)) return 0;
        fq whole = panel(a, b, shift);
        fq tol = 1e-31Q * fabsq(whole);
        if (tol < floor_tol) tol = floor_tol;
        return adapt(a, b, shift, whole, tol, 0);
    }

    /* int_a^inf, by panels 1/|E'(a)| wide past the peak (the decay length) */
    fq integral_to_inf(fq a, fq shift) const
    {
        fq slope = dg * sinhq(a - speak);    /* -E'(a) */
        fq w = (a > speak && slope > 1) ? 1 / slope : 1;
        fq sum = 0;
        for (int k = 0; k < 100000; ++k) {
            fq p = integral(a + k * w, a + (k + 1) * w, shift, 1e-33Q * sum);
            sum += p;
            if (a + k * w > speak && p <= 1e-36Q * sum) break;
        }
        return sum;
    }

    /* f dx = C delta e^{-delta gamma} e^{E(s)} cosh s ds */
    fq log_scale() const { return log_c + logq(delta) - dg; }

    /* log(1 - F(x)), x >= 0 */
    fq log_upper(fq x) const
    {
        fq S = asinhq(x / delta);
        if (S > speak) {
            fq e = E(S);
            return log_scale() + e + logq(integral_to_inf(S, e));
        }
        return log_scale() + logq(integral(S, speak, 0) + integral_to_inf(speak, 0));
    }

    /* log f(x) = log C - (alpha sqrt(delta^2 + x^2) - beta x); for x >= 0 the
       bracket is r x + alpha delta^2 / (sqrt(delta^2 + x^2) + x), r = alpha - beta */
    fq log_f(fq x) const
    {
        fq rt = sqrtq(delta * delta + x * x);
        return log_c - (x >= 0 ? rate * x + alpha * delta * delta / (rt + x) : alpha * rt - beta * x);
    }
};

/* K_1(z) = int_0^inf e^{-z cosh t} cosh t dt, scaled by e^{z} (DLMF 10.32.8) */
fq log_bessel_k1(fq z)
{
    Side k{};
    k.ad = z;
    k.bd = 0;
    k.dg = z;     /* E(t) = -z cosh t + z = -z (cosh t - 1) */
    k.speak = 0;
    return logq(k.integral(0, 1, 0) + k.integral_to_inf(1, 0)) - z;
}

Side make_side(fq alpha, fq beta, fq delta)
{
    Side s{};
    s.alpha = alpha;
    s.beta = beta;
    s.delta = delta;
    s.gamma = sqrtq((alpha - beta) * (alpha + beta));
    s.rate = alpha - beta;
    s.ad = alpha * delta;
    s.bd = beta * delta;
    s.dg = delta * s.gamma;
    s.speak = atanhq(beta / alpha);
    s.log_c = logq(s.gamma / (2 * alpha * delta)) - log_bessel_k1(delta * s.gamma);
    s.log_p = s.log_upper(0);
    return s;
}

/*
 * Taylor coefficients of the right map about v0 from a[0] = Q(v0),
 * a[1] = Q'(v0): with P = Q'^2, S = delta^2 + Q^2, R = S^{-1/2} (Miller:
 * R_k = (1/(k S_0)) sum_{j=1..k} ((1/2) j - k) S_j R_{k-j}) and
 * H = alpha Q R - beta, the power d^k of Q'' + rate Q' = H P gives
 * (k+2)(k+1) a_{k+2} = (H P)_k - rate (k+1) a_{k+1}.
 */
void taylor_step(const Side& sd, fq* a)
{
    fq P[TM + 1], S[TM + 1], R[TM + 1], H[TM + 1];
    for (int k = 0; k + 2 <= TM; ++k) {
        fq p = 0, s2 = 0;
        for (int i = 0; i <= k; ++i) {
            p += (fq)(i + 1) * a[i + 1] * (fq)(k - i + 1) * a[k - i + 1];
            s2 += a[i] * a[k - i];
        }
        P[k] = p;
        S[k] = s2 + (k == 0 ? sd.delta * sd.delta : (fq)0);
        if (k == 0) {
            R[0] = 1 / sqrtq(S[0]);
        } else {
            fq acc = 0;
            for (int j = 1; j <= k; ++j) acc += ((fq)j / 2 - (fq)k) * S[j] * R[k - j];
            R[k] = acc / ((fq)k * S[0]);
        }
        fq qr = 0;
        for (int i = 0; i <= k; ++i) qr += a[i] * R[k - i];
        H[k] = sd.alpha * qr - (k == 0 ? sd.beta : (fq)0);
        fq hp = 0;
        for (int i = 0; i <= k; ++i) hp += H[i] * P[k - i];
        a[k + 2] = (hp - sd.rate * (fq)(k + 1) * a[k + 1]) / ((fq)(k + 2) * (fq)(k + 1));
    }
}

struct Node {
    fq v0, h;
    fq a[TM + 1];
};

fq horner(const fq* a, fq d)
{
    fq r = a[TM];
    for (int k = TM - 1; k >= 0; --k) r = r * d + a[k];
    return r;
}

fq horner_d(const fq* a, fq d)
{
    fq r = TM * a[TM];
    for (int k = TM - 1; k >= 1; --k) r = r * d + k * a[k];
    return r;
}

/* Largest step with the last two Taylor terms below 1e-36 |Q| (at most hmax) */
fq step_size(const fq* a, fq hmax)
{
    fq scale = fabsq(a[0]) + fabsq(a[1]) * 1e-3Q + 1e-300Q, h = hmax;
    for (int k = TM - 1; k <= TM; ++k) {
        if (a[k] == 0) continue;
        fq hk = powq(1e-36Q * scale / fabsq(a[k]), 1.0Q / k);
        if (hk < h) h = hk;
    }
    return h;
}

/* Taylor steps from (v, Q, Q') to v1; false if they do not get there
   within the step budget (the tested parameters need at most a few
   hundred). */
bool integrate(const Side& sd, fq v, fq Q, fq dQ, fq v1, std::vector<Node>& out)
{
    const fq dir = v1 > v ? 1 : -1;
    for (int guard = 0; guard < 20000; ++guard) {
        Node n;
        n.v0 = v;
        n.a[0] = Q;
        n.a[1] = dQ;
        taylor_step(sd, n.a);
        fq hmax = 0.25Q + 0.05Q * fabsq(v);
        fq h = step_size(n.a, hmax);
        bool last = fabsq(v1 - v) <= h;
        if (last) h = fabsq(v1 - v);
        n.h = dir * h;
        out.push_back(n);
        Q = horner(n.a, n.h);
        dQ = horner_d(n.a, n.h);
        v += n.h;
        if (last) return true;
    }
    return false;
}

/*
 * Gauss-Laguerre rule (weight e^{-t} on [0, inf)): the nodes are the
 * eigenvalues of the Jacobi matrix of the Laguerre polynomials (diagonal
 * 2i + 1, off-diagonal i + 1), found one by one by bisection on the Sturm
 * count of negative pivots of J - lambda I; weights
 * w_i = t_i / ((n + 1)^2 L_{n+1}(t_i)^2) (Abramowitz and Stegun 25.4.45).
 */
constexpr int GLAG = 48;

struct Laguerre {
    fq t[GLAG], w[GLAG];
    static int below(fq lam)
    {
        int neg = 0;
        fq d = 1 - lam;
        if (d < 0) ++neg;
        for (int i = 1; i < GLAG; ++i) {
            if (d == 0) d = 1e-60Q;
            d = (2 * i + 1 - lam) - (fq)i * (fq)i / d;
            if (d < 0) ++neg;
        }
        return neg;
    }
    Laguerre()
    {
        for (int i = 0; i < GLAG; ++i) {
            fq lo = 0, hi = 4 * GLAG + 2;
            for (int it = 0; it < 240; ++it) {
                fq mid = (lo + hi) / 2;
                if (below(mid) > i) hi = mid; else lo = mid;
                if (hi - lo <= 1e-33Q * hi) break;
            }
            fq x = (lo + hi) / 2;
            fq p0 = 1, p1 = 1 - x;
            for (int k = 1; k <= GLAG; ++k) {
                fq p2 = ((2 * k + 1 - x) * p1 - k * p0) / (k + 1);
                p0 = p1;
                p1 = p2;
            }
            t[i] = x;
            w[i] = x / ((fq)(GLAG + 1) * (fq)(GLAG + 1) * p1 * p1);
        }
    }
};

const Laguerre& laguerre()
{
    static const Laguerre g;
    return g;
}

/* D = alpha sqrt(delta^2 + x^2) - beta x - delta gamma (the depth below the
   density's peak), with z c0 = r x + alpha delta^2 / (sqrt(delta^2 + x^2) + x)
   formed without cancellation for x >= 0. */
fq depth(const Side& sd, fq x, fq* zc0)
{
    fq rt = sqrtq(sd.delta * sd.delta + x * x);
    fq zc = sd.rate * x + sd.alpha * sd.delta * sd.delta / (rt + x);
    if (zc0) *zc0 = zc;
    return zc - sd.dg;
}

/* log(1 - F(x)) and the ratio m = (1 - F)/f at x past the peak (D large). */
void far_tail(const Side& sd, fq x, fq* log_t, fq* m)
{
    const Laguerre& L = laguerre();
    fq zc0, D = depth(sd, x, &zc0);
    const fq z = sd.dg;
    fq K = 0;
    for (int i = 0; i < GLAG; ++i) {
        fq a = (D + L.t[i]) / z;            /* c - 1 */
        fq ra = sqrtq(a * (a + 2));         /* sqrt(c^2 - 1) */
        K += L.w[i] / (ra * (1 + a + ra));  /* h(c) - 1 */
    }
    fq br = expq(sd.speak) + coshq(sd.speak) * K;
    *log_t = sd.log_c + logq(sd.delta / z) - zc0 + logq(br);
    *m = sd.delta / z * br;
}

constexpr fq D_MIN = 24;   /* Laguerre error ~ e^{-4 sqrt(GLAG D)} << 1e-34 */

/* Q(v) for v past the anchor: Newton on log(1 - F(Q)) = log p - r v, from x0. */
fq solve_far(const Side& sd, fq v, fq x0)
{
    const fq target = sd.log_p - sd.rate * v;
    fq x = x0;
    for (int it = 0; it < 40; ++it) {
        fq lt, m;
        far_tail(sd, x, &lt, &m);
        fq dx = m * (lt - target);
        x += dx;
        if (fabsq(dx) <= 1e-22Q * x) break;     /* the next step would be below 1e-40 */
    }
    return x;
}

/*
 * What the cell fitting needs of one side's map, whatever solves it: Q(v)
 * for v > 0 to far below the cells' tolerance, Q'(0), the side's rate, and
 * the large-v form exactly as the kernel evaluates it,
 *     clog = 0:  Q = v + c0 + (c1 + c2/v)/v,
 *     clog > 0:  Q = v + c0 + clog log Q + (c1 + c2/Q)/Q by three fixed-point
 *                steps from v + c0 + clog log v (tails with a power of x).
 */
struct SideMap {
    fq slope0 = 0, rate = 0;
    fq c0 = 0, c1 = 0, c2 = 0, clog = 0;
    /* rho > 0: the target density carries a factor |x|^rho at 0 with rho not
       an integer (variance-gamma, rho = 2 lambda - 1), so R = Q/v has terms
       in v^(m + n rho) there, which no polynomial cell near v = 0 can match;
       the first octave of cells is then one series in v and v^rho
       (fit_origin) */
    fq rho = 0;
    virtual fq eval(fq v) const = 0;
    virtual ~SideMap() {}
    fq far(fq v) const
    {
        if (clog == 0) return v + c0 + (c1 + c2 / v) / v;
        fq q = v + c0 + clog * logq(v);
        for (int i = 0; i < 3; ++i) q = v + c0 + clog * logq(q) + (c1 + c2 / q) / q;
        return q;
    }
};

/* The solution of one side: ODE legs on [0, v_a], direct solves beyond. */
struct SideSolution : SideMap {
    const Side* sd;
    std::vector<Node> fwd, bwd;
    fq v_match, v_a;

    fq eval(fq v) const override
    {
        if (v > v_a) return solve_far(*sd, v, far(v));
        const std::vector<Node>& nd = v <= v_match ? fwd : bwd;
        /* fwd nodes increase in v0, bwd nodes decrease */
        size_t lo = 0, hi = nd.size() - 1;
        const bool up = nd.front().h > 0;
        while (lo < hi) {
            size_t mid = (lo + hi) / 2;
            fq a = nd[mid].v0, b = nd[mid].v0 + nd[mid].h;
            fq lo_v = up ? a : b, hi_v = up ? b : a;
            if (v < lo_v) {
                if (up) hi = mid; else lo = mid + 1;
            } else if (v > hi_v) {
                if (up) lo = mid + 1; else hi = mid;
            } else {
                lo = hi = mid;
            }
        }
        return horner(nd[lo].a, v - nd[lo].v0);
    }
};

int fail(char* err, int errlen, const char* msg)
{
    snprintf(err, errlen, "%s", msg);
    return -1;
}

/* Chebyshev interpolant of fv (values at the K+1 Chebyshev points of
   [c - hw, c + hw]) as monomials in d = v - c. */
void cheb_to_monomial(const fq* fv, int K, fq hw, fq* mono)
{
    const int N = K + 1;
    fq ck[64], Tp[64], Tc[64], Tn[64];
    for (int j = 0; j < N; ++j) {
        fq s = 0;
        for (int i = 0; i < N; ++i) s += fv[i] * cosq(M_PIq * j * (i + 0.5Q) / N);
        ck[j] = s * 2 / N;
    }
    ck[0] /= 2;
    for (int i = 0; i < N; ++i) {
        mono[i] = 0;
        Tp[i] = 0;
        Tc[i] = 0;
    }
    Tp[0] = 1;
    Tc[1] = 1;
    for (int i = 0; i < N; ++i) mono[i] += ck[0] * Tp[i] + ck[1] * Tc[i];
    for (int j = 2; j < N; ++j) {
        for (int i = 0; i < N; ++i) Tn[i] = -Tp[i] + (i > 0 ? 2 * Tc[i - 1] : (fq)0);
        for (int i = 0; i < N; ++i) mono[i] += ck[j] * Tn[i];
        memcpy(Tp, Tc, sizeof(fq) * N);
        memcpy(Tc, Tn, sizeof(fq) * N);
    }
    fq sc = 1;
    for (int i = 0; i < N; ++i) {
        mono[i] /= sc;
        sc *= hw;
    }
}

/*
 * Large-v form.  With phi = log f - log C = -alpha sqrt(delta^2 + x^2) + beta x
 * = -r x - alpha delta^2/(2x) + O(x^-3) (r = alpha - beta), the tail mass is
 * T = C e^phi / (-phi') (1 + O(phi''/phi'^2)) with -phi' = r - alpha delta^2/(2x^2)
 * + O(x^-4) and phi'' = O(x^-3), so log T = log(C/r) - r x - a/x + a/(r x^2)
 * + O(x^-3), a = alpha delta^2 / 2.  Solving log T(Q) = log p - r v for Q
 * and expanding 1/Q gives c0 = log(C/(r p))/r, c1 = -a/r,
 * c2 = (a/r)(c0 + 1/r).
 */
bool solve_side(const Side& sd, SideSolution* ss, char* err, int errlen)
{
    const fq r = sd.rate;
    ss->sd = &sd;
    ss->rate = r;
    ss->c0 = (sd.log_c - logq(r) - sd.log_p) / r;
    const fq a = sd.alpha * sd.delta * sd.delta / 2;
    ss->c1 = -a / r;
    ss->c2 = (a / r) * (ss->c0 + 1 / r);
    ss->slope0 = expq(sd.log_p - sd.log_f(0)) * r;
    /* the anchor: far enough for the forward leg to stop at 20/r and for
       the direct solve to be accurate (D >= D_MIN) */
    fq va = 40 / r;
    for (int it = 0; it < 200; ++it) {
        fq x = solve_far(sd, va, ss->far(va) > 0 ? ss->far(va) : va);
        if (depth(sd, x, nullptr) >= D_MIN && x > 0) break;
        va *= 1.25Q;
    }
    ss->v_a = va;
    ss->v_match = 20 / r;
    const fq Qa = solve_far(sd, va, ss->far(va));
    const fq dQa = expq(sd.log_p - r * va + logq(r) - sd.log_f(Qa));
    if (!integrate(sd, 0, 0, ss->slope0, ss->v_match, ss->fwd) ||
        !integrate(sd, va, Qa, dQa, ss->v_match, ss->bwd)) {
        snprintf(err, errlen, "the ODE integration exceeded its step budget");
        return false;
    }
    const Node& f = ss->fwd.back();
    const Node& b = ss->bwd.back();
    fq qf = horner(f.a, f.h), qb = horner(b.a, b.h);
    fq df = horner_d(f.a, f.h), db = horner_d(b.a, b.h);
    fq mis = fabsq(qf / qb - 1) + fabsq(df / db - 1);
    if (!(mis < 1e-19Q)) {   /* two orders below the cells' 2e-17 */
        snprintf(err, errlen, "legs disagree at v=%g by %.3e", (double)ss->v_match, (double)mis);
        return false;
    }
    return true;
}

/* The smallest power of 2, P, from which on the large-v form meets tol
   (checked on [P, 3P]). */
bool far_start(const SideMap& ss, fq tol, fq* P)
{
    fq p = ldexpq(1, (int)ceilq(log2q(ldexpq(1, 30) / ss.rate)));
    auto holds = [&](fq q) {
        for (int i = 0; i <= 16; ++i) {
            fq v = q * (1 + (fq)i / 8);
            if (fabsq(ss.far(v) / ss.eval(v) - 1) > tol) return false;
        }
        return true;
    };
    if (!holds(p)) return false;
    while (p > ldexpq(1, -40) && holds(p / 2)) p /= 2;
    *P = p;
    return true;
}

/*
 * Fit R = Q/v on [lo, hi] (degree deg, Chebyshev points), rounded to
 * double, highest power first.  Returns the largest relative error of the
 * interpolant at 2 deg + 1 points against the solution; *rounded gets that
 * of the double row (which includes the rounding of R itself).
 */
fq fit_cell(const SideMap& ss, int deg, fq lo, fq hi, double* row, fq* rounded)
{
    fq c = (lo + hi) / 2, hw = (hi - lo) / 2;
    fq fv[64], mono[64];
    for (int i = 0; i <= deg; ++i) {
        fq v = c + hw * cosq(M_PIq * (i + 0.5Q) / (deg + 1));
        fv[i] = ss.eval(v) / v;
    }
    cheb_to_monomial(fv, deg, hw, mono);
    for (int k = 0; k <= deg; ++k) row[deg - k] = (double)mono[k];
    fq worst = 0, worst_r = 0, share = 0;
    const int NT = 2 * deg;
    for (int t = 0; t <= NT; ++t) {
        fq d = -hw + 2 * hw * t / NT;
        fq v = c + d;
        fq ref = v > 0 ? ss.eval(v) / v : ss.slope0;
        fq pe = 0, pr = 0;
        for (int k = deg; k >= 0; --k) pe = pe * d + mono[k];
        for (int k = 0; k <= deg; ++k) pr = pr * d + (fq)row[k];
        fq et = fabsq(pe / ref - 1), er = fabsq(pr / ref - 1);
        if (et > worst) worst = et;
        if (er > worst_r) worst_r = er;
        fq sh = fabsq((pe - mono[0]) / ref);
        if (sh > share) share = sh;
    }
    /* the FP32-output cells are evaluated as c0 + d S(d) with S in FP32
       (qm_hyp_device.hpp), which needs the non-constant part to stay a small
       share of R: a cell where it exceeds 1/8 counts as missing the target */
    if (deg == HYP_DEGREE_F32 && share > 0.125Q) worst = 1;
    *rounded = worst_r;
    return worst;
}

/* Bounds in v of cell j = HYP_SUB k + i: t = 1 + v/v0 in
   [2^k (1 + i/S), 2^k (1 + (i+1)/S)). */
void cell_bounds(fq v0, int j, fq* lo, fq* hi)
{
    const int k = j / HYP_SUB, i = j % HYP_SUB;
    *lo = v0 * (ldexpq(1 + (fq)i / HYP_SUB, k) - 1);
    *hi = v0 * (ldexpq(1 + (fq)(i + 1) / HYP_SUB, k) - 1);
}

/* One cell set: its degree and the truncation tolerance its cells meet. */
struct CellSpec {
    int deg;
    fq tol;
};

/* Host threads for fitting cells: the cells are independent and each one
   only reads the side's solution. */
int fit_threads()
{
    static const int n = [] {
        const char* e = getenv("QM_BUILD_THREADS");
        long v = e ? strtol(e, nullptr, 10) : (long)std::thread::hardware_concurrency();
        return (int)(v < 1 ? 1 : (v > 16 ? 16 : v));
    }();
    return n;
}

/* Fit cells [j0, j1) of a side for v0 into rows (deg + 1 doubles per cell,
   cell j0 first), on up to fit_threads() threads.  Returns false, with the
   first failing cell in *bad, if one misses tol; *worst gets the largest
   error of the rounded rows. */
bool fit_cells(const SideMap& ss, const CellSpec& cs, fq v0, int j0, int j1, double* rows, fq* worst, int* bad)
{
    const int W = cs.deg + 1, count = j1 - j0;
    if (count <= 0) return true;
    std::vector<fq> err(count), rerr(count);
    auto work = [&](int first, int step) {
        for (int i = first; i < count; i += step) {
            fq lo, hi;
            cell_bounds(v0, j0 + i, &lo, &hi);
            err[i] = fit_cell(ss, cs.deg, lo, hi, rows + (size_t)i * W, &rerr[i]);
        }
    };
    const int T = count < fit_threads() ? count : fit_threads();
    if (T <= 1) {
        work(0, 1);
    } else {
        std::vector<std::thread> pool;
        for (int t = 1; t < T; ++t) pool.emplace_back(work, t, T);
        work(0, T);
        for (auto& th : pool) th.join();
    }
    for (int i = 0; i < count; ++i) {
        if (rerr[i] > *worst) *worst = rerr[i];
        if (err[i] > cs.tol) {
            *bad = j0 + i;
            return false;
        }
    }
    return true;
}

/*
 * The first octave of t (v in [0, v0)) of a side with rho > 0, as one
 * series in v and w = v^rho (the terms v^(m + n rho) of R near the origin):
 *     R = P0(v) + w (P1(v) + w (P2(v) + w P3(v))),
 * P0..P3 of degrees 4, 2, 1, 0 for the FP64-output cells (row of 12
 * doubles: rho, then the coefficients of P3, P2, P1 and P0, each highest
 * power first) and P0..P2 of degrees 3, 1, 0 for the FP32-output cells
 * (row of 8).  The smallest exponent left out is at least 4 (3 for FP32
 * outputs), since rho > 1.  Where two terms have the same exponent (rho a
 * fraction such as 3/2: v^3 and w^2), or exponents within 1e-9, the term
 * of the higher family is left out (its coefficient is 0).  Fitted by
 * least squares (Householder QR, in __float128) on Chebyshev nodes of
 * s = v/v0 in [0, 1], in the scaled basis s^(m + n rho), then checked like
 * a cell, as the kernel evaluates it (w = v^rho rounded to a double, the
 * row's rounded coefficients), on a uniform and a geometric grid down to
 * v = v0 1e-30.  Returns the worst truncation error; *rounded gets that of
 * the rounded row.
 */
constexpr int ORIGIN_DEG64[4] = {4, 2, 1, 0};
constexpr int ORIGIN_DEG32[3] = {3, 1, 0};

fq fit_origin(const SideMap& ss, int deg, fq v0, double* row, fq* rounded)
{
    const bool f64 = deg == HYP_DEGREE;
    const int nfam = f64 ? 4 : 3;
    const int* dg = f64 ? ORIGIN_DEG64 : ORIGIN_DEG32;
    const fq rho = (fq)(double)ss.rho;           /* the kernel's rho */
    int pw_m[16], pw_n[16], K = 0;
    for (int n = nfam - 1; n >= 0; --n)
        for (int m = dg[n]; m >= 0; --m) {
            pw_m[K] = m;
            pw_n[K] = n;
            ++K;
        }
    /* the fitted terms: all but those whose exponent a lower family has */
    int col[16], J = 0;
    for (int k = 0; k < K; ++k) {
        bool dup = false;
        for (int l = 0; l < K; ++l)
            if (pw_n[l] < pw_n[k] && fabsq(pw_m[l] + pw_n[l] * rho - (pw_m[k] + pw_n[k] * rho)) < 1e-9Q) dup = true;
        if (!dup) col[J++] = k;
    }
    /* least squares: A a = f, A_ij = s_i^(m_k + n_k rho), k = col[j] */
    const int N = 4 * K;
    std::vector<fq> A((size_t)N * J), f(N);
    for (int i = 0; i < N; ++i) {
        const fq sn = (1 - cosq(M_PIq * (i + 0.5Q) / N)) / 2;
        const fq v = v0 * sn;
        f[i] = ss.eval(v) / v;
        for (int j = 0; j < J; ++j) A[(size_t)i * J + j] = powq(sn, pw_m[col[j]] + pw_n[col[j]] * rho);
    }
    /* Householder QR applied to [A | f] */
    for (int k = 0; k < J; ++k) {
        fq nrm = 0;
        for (int i = k; i < N; ++i) nrm += A[(size_t)i * J + k] * A[(size_t)i * J + k];
        nrm = sqrtq(nrm);
        const fq akk = A[(size_t)k * J + k];
        const fq alpha = akk > 0 ? -nrm : nrm;
        std::vector<fq> u(N, 0);
        u[k] = akk - alpha;
        for (int i = k + 1; i < N; ++i) u[i] = A[(size_t)i * J + k];
        fq uu = 0;
        for (int i = k; i < N; ++i) uu += u[i] * u[i];
        if (uu == 0) continue;
        for (int j = k; j < J; ++j) {
            fq d = 0;
            for (int i = k; i < N; ++i) d += u[i] * A[(size_t)i * J + j];
            d = 2 * d / uu;
            for (int i = k; i < N; ++i) A[(size_t)i * J + j] -= d * u[i];
        }
        fq d = 0;
        for (int i = k; i < N; ++i) d += u[i] * f[i];
        d = 2 * d / uu;
        for (int i = k; i < N; ++i) f[i] -= d * u[i];
    }
    std::vector<fq> a(J);
    for (int k = J - 1; k >= 0; --k) {
        fq t = f[k];
        for (int j = k + 1; j < J; ++j) t -= A[(size_t)k * J + j] * a[j];
        a[k] = t / A[(size_t)k * J + k];
    }
    /* unscaled coefficients of v^m w^n, the row as the kernel reads it */
    fq c[16];
    for (int k = 0; k < K; ++k) c[k] = 0;
    for (int j = 0; j < J; ++j) c[col[j]] = a[j] / powq(v0, pw_m[col[j]] + pw_n[col[j]] * rho);
    row[0] = (double)rho;
    for (int k = 0; k < K; ++k) row[1 + k] = (double)c[k];
    auto eval = [&](fq v, fq w, bool use_row) {
        /* Horner in v within each family, then in w, highest family first */
        fq R = 0;
        int k = 0;
        for (int n = nfam - 1; n >= 0; --n) {
            fq p = 0;
            for (int m = dg[n]; m >= 0; --m, ++k) p = p * v + (use_row ? (fq)row[1 + k] : c[k]);
            R = R * w + p;
        }
        return R;
    };
    fq worst = 0, worst_r = 0;
    for (int t = 0; t <= 400; ++t) {
        const fq v = t <= 200 ? v0 * t / 200 : v0 * powq(10, -30 * (fq)(t - 201) / 199);
        const fq ref = v > 0 ? ss.eval(v) / v : ss.slope0;
        const fq w = powq(v, rho);
        const fq wd = (fq)(double)powq((fq)(double)v, rho);
        const fq et = fabsq(eval(v, w, false) / ref - 1), er = fabsq(eval((fq)(double)v, wd, true) / ref - 1);
        if (et > worst) worst = et;
        if (er > worst_r) worst_r = er;
    }
    *rounded = worst_r;
    return worst;
}

/*
 * Cells of one side for v0 = 2^lv, lv <= max_lv: the largest lv whose
 * cells all meet the tolerance (the first octave of t, uniform cells on
 * [0, v0), and the next two decide it; the rest are then fitted and
 * checked).  The cells reach v_top = v0 (2^noct - 1), beyond the first
 * power of 2 from which on the large-v form holds to a quarter of the
 * tolerance.  Returns lv, or INT_MIN with a message if none fits.
 */
int fit_side(const SideMap& ss, const CellSpec& cs, int max_lv, std::vector<double>* rows_out, HypSide* hs,
             char* err, int errlen)
{
    fq P;
    if (!far_start(ss, cs.tol / 4, &P)) {
        snprintf(err, errlen, "large-v form not accurate at 2^30 / (alpha - beta)");
        return INT_MIN;
    }
    const int W = cs.deg + 1;
    int lv = (int)lrintq(log2q(P));
    if (lv > 3) lv = 3;
    if (lv > max_lv) lv = max_lv;
    for (; lv >= -60; --lv) {
        const fq v0 = ldexpq(1, lv);
        int noct = 1;
        while (v0 * (ldexpq(1, noct) - 1) < P) ++noct;
        if (noct > HYP_MAX_OCT) break;
        const int ncell = HYP_SUB * noct;
        std::vector<double> rows((size_t)ncell * W);
        fq worst = 0;
        int bad = -1;
        const int head = ncell < 3 * HYP_SUB ? ncell : 3 * HYP_SUB;
        const bool origin = ss.rho > 0;
        if (origin) {
            /* the first octave: one series in v and v^rho in row 0 (rows 1..7
               are not read); the cells from the second octave on as usual */
            fq ow = 0;
            if (fit_origin(ss, cs.deg, v0, rows.data(), &ow) > cs.tol || !(ow < 6 * cs.tol + 1.2e-16Q)) continue;
            if (ow > worst) worst = ow;
            if (!fit_cells(ss, cs, v0, HYP_SUB, head, rows.data() + (size_t)HYP_SUB * W, &worst, &bad)) continue;
        } else if (!fit_cells(ss, cs, v0, 0, head, rows.data(), &worst, &bad)) {
            continue;
        }
        if (!fit_cells(ss, cs, v0, head, ncell, rows.data() + (size_t)head * W, &worst, &bad)) {
            fq lo, hi;
            cell_bounds(v0, bad, &lo, &hi);
            snprintf(err, errlen, "cell near v=%g misses the accuracy target", (double)lo);
            return INT_MIN;
        }
        hs->v0 = (double)v0;
        hs->inv_v0 = (double)(1 / v0);
        hs->v_top = (double)(v0 * (ldexpq(1, noct) - 1));
        hs->far_c0 = (double)ss.c0;
        hs->far_c1 = (double)ss.c1;
        hs->far_c2 = (double)ss.c2;
        hs->far_clog = (double)ss.clog;
        hs->max_rel_err = (double)worst;
        hs->noct = noct;
        hs->ncell = ncell;
        hs->degree = cs.deg;
        hs->origin = origin ? 1 : 0;
        *rows_out = std::move(rows);
        return lv;
    }
    snprintf(err, errlen, "no cell width met the accuracy target within %d octaves", HYP_MAX_OCT);
    return INT_MIN;
}

/* Both sides' cells of one set, with one v0: the smaller of the two sides'
   own choices.  Appends the right side's rows, then the left side's. */
bool fit_set(const SideMap& rs, const SideMap& ls, const CellSpec& cs, HypSide* right, HypSide* left,
             std::vector<double>& coef, char* err, int errlen)
{
    std::vector<double> rr, rl;
    int lr = fit_side(rs, cs, 3, &rr, right, err, errlen);
    if (lr == INT_MIN) return false;
    int ll = fit_side(ls, cs, lr, &rl, left, err, errlen);
    for (int it = 0; it < 8 && ll != INT_MIN && ll != lr; ++it) {
        lr = fit_side(rs, cs, ll, &rr, right, err, errlen);
        if (lr == INT_MIN) return false;
        if (lr != ll) ll = fit_side(ls, cs, lr, &rl, left, err, errlen);
    }
    if (ll == INT_MIN) return false;
    if (ll != lr) {
        snprintf(err, errlen, "no common cell width");
        return false;
    }
    right->coef_offset = coef.size();
    coef.insert(coef.end(), rr.begin(), rr.end());
    left->coef_offset = coef.size();
    coef.insert(coef.end(), rl.begin(), rl.end());
    return true;
}

bool check_params(double alpha, double beta, double delta)
{
    return std::isfinite(alpha) && std::isfinite(beta) && std::isfinite(delta) && delta > 0 &&
           alpha > std::fabs(beta);
}

/*
 * Variance-gamma sides (Section 8.2) for integer lambda = n + 1.  Then
 * K_{n+1/2}(z) = sqrt(pi/(2z)) e^{-z} sum_{k<=n} (n+k)!/(k!(n-k)!) (2z)^{-k}
 * (DLMF 10.49.12), so on the side's half-line the density is
 * A e^{-r x} sum_m d_m x^m and the tail mass A e^{-r x} sum_j t_j x^j, both
 * with positive coefficients, and Q(v) comes from the defining equation
 * directly: Newton on the central mass int_0^x f = p (1 - e^{-r v}) (the
 * lower incomplete gamma series, no cancellation) while r v <= ln 2, on
 * log(1 - F) = log p - r v beyond.  No ODE is needed; the large-v form is
 * the log one: log(1 - F(x)) = log(A t_n) - r x + n log x + log(1 + s1/x + s2/x^2 + ...),
 * s_i = t_{n-i}/t_n, so Q = v + c0 + (n/r) log Q + (s1/Q + (s2 - s1^2/2)/Q^2)/r + O(Q^-3).
 */
constexpr int VG_LAMBDA_MAX = 8;

struct VGSide : SideMap {
    int n;
    fq logA, log_p;
    fq c[VG_LAMBDA_MAX], tp[VG_LAMBDA_MAX], dp[VG_LAMBDA_MAX];

    static fq fact(int k) { return expq(lgammaq((fq)k + 1)); }
    static fq poly(const fq* a, int deg, fq x)
    {
        fq r = a[deg];
        for (int j = deg - 1; j >= 0; --j) r = r * x + a[j];
        return r;
    }
    fq log_tail(fq x) const { return logA - rate * x + logq(poly(tp, n, x)); }
    fq log_dens(fq x) const { return logA - rate * x + logq(poly(dp, n, x)); }

    /* int_0^x t^m e^{-r t} dt */
    fq lower(int m, fq x) const
    {
        const fq y = rate * x;
        const fq full = fact(m) / powq(rate, m + 1);
        if (y > m + 60) {
            fq term = 1, sum = 1;
            for (int j = 1; j <= m; ++j) {
                term *= y / j;
                sum += term;
            }
            return full * (1 - expq(-y) * sum);
        }
        fq term = expq(-y), sum = 0;
        for (int j = 1; j <= m; ++j) term *= y / j;
        for (int j = m + 1; j < 100000; ++j) {
            term *= y / j;
            sum += term;
            if (term <= 1e-36Q * sum) break;
        }
        return full * sum;
    }
    fq central_mass(fq x) const
    {
        fq sum = 0;
        for (int k = 0; k <= n; ++k) sum += c[k] * lower(n - k, x);
        return expq(logA) * sum;
    }

    VGSide(int n_, fq alpha, fq beta) : n(n_)
    {
        rate = alpha - beta;
        const fq lam = n + 1;
        logA = lam * logq((alpha - beta) * (alpha + beta)) + logq(sqrtq(M_PIq / (2 * alpha))) -
               (lam - 0.5Q) * logq(2 * alpha) - 0.5Q * logq(M_PIq) - lgammaq(lam);
        for (int k = 0; k <= n; ++k)
            c[k] = expq(lgammaq((fq)(n + k) + 1) - lgammaq((fq)k + 1) - lgammaq((fq)(n - k) + 1) - k * logq(2 * alpha));
        for (int m = 0; m <= n; ++m) dp[m] = c[n - m];
        for (int j = 0; j <= n; ++j) {
            fq t = 0;
            for (int k = 0; k <= n - j; ++k) t += c[k] * fact(n - k) / (fact(j) * powq(rate, n - k - j + 1));
            tp[j] = t;
        }
        log_p = log_tail(0);
        slope0 = expq(log_p - log_dens(0)) * rate;
        c0 = (logA + logq(tp[n]) - log_p) / rate;
        clog = (fq)n / rate;
        const fq s1 = n >= 1 ? tp[n - 1] / tp[n] : 0, s2 = n >= 2 ? tp[n - 2] / tp[n] : 0;
        c1 = s1 / rate;
        c2 = (s2 - s1 * s1 / 2) / rate;
    }

    fq eval(fq v) const override
    {
        const fq a = rate * v;
        fq x;
        if (a <= M_LN2q) {
            const fq target = -expq(log_p) * expm1q(-a);
            x = slope0 * v;
            for (int it = 0; it < 200; ++it) {
                fq dx = (central_mass(x) - target) / expq(log_dens(x));
                fq xn = x - dx;
                if (!(xn > 0)) xn = x / 2;
                if (fabsq(xn - x) <= 1e-33Q * xn) return xn;
                x = xn;
            }
            return x;
        }
        const fq target = log_p - a;
        x = v + c0 + (clog > 0 ? clog * logq(v) : (fq)0);
        if (!(x > 0)) x = v;
        for (int it = 0; it < 200; ++it) {
            fq lt = log_tail(x);
            fq xn = x + (lt - target) * expq(lt - log_dens(x));
            if (!(xn > 0)) xn = x / 2;
            if (fabsq(xn - x) <= 1e-33Q * xn) return xn;
            x = xn;
        }
        return x;
    }
};

/*
 * Variance-gamma sides (Section 8.2) for real lambda in (1, 8]: the
 * recycling ODE, as the paper prescribes ("solved as before"),
 *     Q'' + r Q' = H(Q) Q'^2,  H(x) = alpha K_{nu-1}(alpha x)/K_nu(alpha x) - beta,
 * r = alpha - beta, nu = lambda - 1/2 (Section 8.2 gives H).  Two pieces of
 * analysis carry it:
 *
 * The Bessel ratio R(z) = K_{nu-1}(z)/K_nu(z).  From K'_nu = -K_{nu-1} - (nu/z) K_nu
 * and K'_{nu-1} = -K_nu + ((nu-1)/z) K_{nu-1} (DLMF 10.29.2), R solves the
 * Riccati equation R' = R^2 + (2 nu - 1) R / z - 1, and L(z) = log(z^nu K_nu(z)) + z
 * solves L' = 1 - R.  Both are integrated by the Taylor-series method
 * backwards from z = 45, where the large-z expansion
 *     K_mu(z) ~ sqrt(pi/(2z)) e^{-z} sum_k a_k(mu) z^{-k},
 *     a_k = a_{k-1} (4 mu^2 - (2k-1)^2) / (8k)     (DLMF 10.40.2)
 * is good to e^{-2z}, down to z = 1e-30: backwards R is the decaying
 * (minimal) solution, so errors shrink.  The build checks L near 0 against
 * its exact limit log(2^{nu-1} Gamma(nu)).  The density is then
 *     log f(x) = log A - nu log alpha + L(alpha x) - r x.
 *
 * The origin.  For non-integer lambda the density has a term in x^{2 lambda - 1}
 * at 0, so Q is not analytic at v = 0 (the paper leaves these cases to an
 * analytical estimate in a small neighbourhood of the origin, the numerical
 * solution starting a small distance away).  Here that estimate is
 * Q = Q'(0) v + Q''(0) v^2 / 2, Q''(0) = -r Q'(0) - beta Q'(0)^2 (H(0) = -beta
 * for lambda > 1), whose remainder is O(v^2, v^{2 lambda - 1}) relative;
 * it holds to 1e-34 below v_min = min(1e-17, 10^{-34/(2 lambda - 1)}).  A
 * leg starts there and runs forwards, with steps growing with v, to
 * v_s = 1/(8 max(1, r)), where it must agree with a direct solve of
 * int_0^Q f = p (1 - e^{-r v_s}) (Gauss-Legendre on panels halving towards
 * 0).  (Integrated towards 0 instead, the ODE's translation mode, an
 * absolute shift of Q(v + d), would turn rounding into a relative error d/v
 * that grows without bound.)
 *
 * As for the hyperbolic target, a forward leg from v_s meets, at
 * v = 20/r, a backward leg from an anchor where Q solves the tail
 * condition log(1 - F(Q)) = log p - r v_a directly (Gauss-Laguerre in
 * the distance past Q, exact for the tail's slowly varying factor once
 * r Q >= 24), and Q is that direct solve beyond the anchor.  In v the
 * system is Q' = P, P' = -r P + (alpha R - beta) P^2,
 * R' = alpha P (R^2 - 1) + (2 nu - 1) R P / Q; forwards in z the Riccati
 * equation is unstable (its dominant solutions are I-type), so every
 * step takes R(alpha Q) afresh from the backward Bessel solution and the
 * recurrence only supplies its higher Taylor coefficients.
 *
 * The masses are the paper's closed form (A&S 6.621.3), with the Pfaff
 * transformation 2F1(a, b; c; z) = (1 - z)^{-b} 2F1(c - a, b; c; z/(z - 1))
 * (DLMF 15.8.1) turning it into a series in w = (1 + beta/alpha)/2 < 1:
 *     p+ = 2^{lambda-1} (1 + beta/alpha)^lambda Gamma(lambda + 1/2)
 *          2F1(1 - lambda, lambda; lambda + 1; w) / (sqrt(pi) Gamma(lambda + 1));
 * the build checks them against quadrature of f.  The large-v form is the
 * log one, from K_nu's expansion: 1 - F(x) ~ (A sqrt(pi/(2 alpha))/r)
 * e^{-r x} x^{lambda-1} (1 + s1/x + s2/x^2), s1 = (lambda - 1)/r + e1,
 * s2 = (lambda - 1)(lambda - 2)/r^2 + e1 (lambda - 2)/r + e2, e_k = a_k(nu)/alpha^k.
 */
struct BesselRatio {
    struct Node {
        fq z0, h;
        fq R[TM + 1], L[TM + 1];
    };
    fq nu = 0;
    fq z_big = 45, z_min = 1e-30Q;
    fq L0 = 0;                 /* log(2^{nu-1} Gamma(nu)), the limit of L at 0 */
    std::vector<Node> nodes;   /* z decreasing */

    static fq series(fq mu, fq z)
    {
        fq a = 1, sum = 1;
        for (int k = 1; k < 200; ++k) {
            fq an = a * (4 * mu * mu - (fq)(2 * k - 1) * (fq)(2 * k - 1)) / (8 * k * z);
            if (fabsq(an) >= fabsq(a) && k > 1) break;   /* past the smallest term */
            a = an;
            sum += a;
            if (fabsq(a) <= 1e-38Q * fabsq(sum)) break;
        }
        return sum;
    }
    void asym(fq z, fq* R, fq* L) const
    {
        const fq sn = series(nu, z);
        *R = series(nu - 1, z) / sn;
        *L = nu * logq(z) + 0.5Q * logq(M_PIq / (2 * z)) + logq(sn);
    }
    /* Taylor coefficients of R and L about z0 from R[0], L[0] */
    void step(Node& n) const
    {
        fq W[TM + 1], RR[TM + 1], RW[TM + 1];
        for (int k = 0; k <= TM; ++k) W[k] = (k % 2 ? -1 : 1) / powq(n.z0, k + 1);   /* 1/z */
        for (int k = 0; k < TM; ++k) {
            fq rr = 0, rw = 0;
            for (int i = 0; i <= k; ++i) {
                rr += n.R[i] * n.R[k - i];
                rw += n.R[i] * W[k - i];
            }
            RR[k] = rr;
            RW[k] = rw;
            n.R[k + 1] = (RR[k] + (2 * nu - 1) * RW[k] - (k == 0 ? 1 : 0)) / (k + 1);
            n.L[k + 1] = ((k == 0 ? 1 : 0) - n.R[k]) / (k + 1);
        }
    }
    bool build(fq nu_, char* err, int errlen)
    {
        nu = nu_;
        L0 = (nu - 1) * M_LN2q + lgammaq(nu);
        Node n;
        n.z0 = z_big;
        asym(z_big, &n.R[0], &n.L[0]);
        for (int guard = 0; guard < 100000; ++guard) {
            step(n);
            fq scale = fabsq(n.R[0]) + fabsq(n.L[0]) + 1e-300Q, h = n.z0 / 4;
            for (int k = TM - 1; k <= TM; ++k) {
                fq m = fabsq(n.R[k]) + fabsq(n.L[k]);
                if (m == 0) continue;
                fq hk = powq(1e-36Q * scale / m, 1.0Q / k);
                if (hk < h) h = hk;
            }
            const bool last = n.z0 - h <= z_min;
            if (last) h = n.z0 - z_min;
            n.h = -h;
            nodes.push_back(n);
            Node m;
            m.z0 = n.z0 - h;
            m.R[0] = horner(n.R, n.h);
            m.L[0] = horner(n.L, n.h);
            n = m;
            if (last) {
                /* L(z) - z tends to log(2^{nu-1} Gamma(nu)); at 1e-30 the
                   remaining terms are O(z^{min(2 nu, 2)} log z) */
                if (!(fabsq(m.L[0] - m.z0 - L0) < 1e-28Q)) {
                    snprintf(err, errlen, "Bessel ratio integration missed its limit at 0 by %.3e",
                             (double)fabsq(m.L[0] - m.z0 - L0));
                    return false;
                }
                return true;
            }
        }
        snprintf(err, errlen, "Bessel ratio integration exceeded its step budget");
        return false;
    }
    /* R(z) and L(z) for z > 0 */
    void eval(fq z, fq* R, fq* L) const
    {
        if (z >= z_big) {
            asym(z, R, L);
            return;
        }
        if (z <= z_min) {            /* z^nu K_nu -> 2^{nu-1} Gamma(nu); R -> 0 (nu > 1/2) */
            *R = 0;
            *L = L0 + z;
            return;
        }
        size_t lo = 0, hi = nodes.size() - 1;     /* node with z0 + h <= z <= z0 */
        while (lo < hi) {
            size_t mid = (lo + hi) / 2;
            if (z < nodes[mid].z0 + nodes[mid].h) lo = mid + 1; else hi = mid;
        }
        const Node& n = nodes[lo];
        *R = horner(n.R, z - n.z0);
        *L = horner(n.L, z - n.z0);
    }
};

struct VGRealSide : SideMap {
    struct VNode {
        fq v0, h;
        fq Q[TM + 1], P[TM + 1];
    };
    fq lambda, nu, alpha, beta;
    fq logA, log_p, log_f0, q2;
    BesselRatio bes;
    std::vector<VNode> zero, fwd, bwd;     /* legs: v_min -> v_s, v_s -> v_match, v_a -> v_match */
    fq v_min, v_s, v_match, v_a;

    fq log_f(fq x) const
    {
        fq R, L;
        bes.eval(alpha * x, &R, &L);
        return logA - nu * logq(alpha) + L - rate * x;
    }
    /* int_0^x f by 24-point Gauss-Legendre on [x/2^{k+1}, x/2^k], k < 120 (the
       panels keep the x^{2 lambda - 1} term at 0 a panel-width away), plus
       f(0) times the rest */
    fq central_mass(fq x) const
    {
        const GL& g = gl();
        fq sum = 0;
        fq b = x;
        for (int k = 0; k < 120; ++k) {
            const fq a = b / 2, c = (a + b) / 2, r = (b - a) / 2;
            fq p = 0;
            for (int i = 0; i < GLN; ++i) p += g.w[i] * expq(log_f(c + r * g.x[i]));
            sum += p * r;
            b = a;
        }
        return sum + expq(log_f0) * b;
    }
    /* log(1 - F(x)) far out (r x >= 80, alpha x >= 45): with K_nu's expansion
       f(t) = A sqrt(pi/(2 alpha)) t^{lambda-1} e^{-r t} sum_j e_j t^{-j},
       e_j = a_j(nu) alpha^{-j}, and int_x^inf t^mu e^{-r t} dt =
       e^{-r x} x^mu / r sum_m mu (mu - 1) ... (mu - m + 1) (r x)^{-m}, both
       asymptotic series good to e^{-min(2 alpha x, r x)} < 1e-34 here. */
    fq log_tail_far(fq x) const
    {
        fq B = 0, e = 1;
        for (int j = 0; j < 200; ++j) {
            if (j > 0) {
                const fq en = e * (4 * nu * nu - (fq)(2 * j - 1) * (fq)(2 * j - 1)) / (8 * j * alpha * x);
                if (fabsq(en) >= fabsq(e) && j > 1) break;
                e = en;
            }
            const fq mu = lambda - 1 - j;
            fq term = e, inner = 0;
            for (int m = 0; m < 400; ++m) {
                inner += term;
                const fq tn = term * (mu - m) / (rate * x);
                if (fabsq(tn) >= fabsq(term) && m > 0) break;
                term = tn;
                if (fabsq(term) <= 1e-38Q * fabsq(B + inner)) break;
            }
            B += inner;
            if (fabsq(e) <= 1e-38Q * fabsq(B)) break;
        }
        return logA + 0.5Q * logq(M_PIq / (2 * alpha)) - logq(rate) - rate * x + (lambda - 1) * logq(x) + logq(B);
    }
    /* log(1 - F(x)) for r x >= 24: with t = x + u/r,
       1 - F(x) = e^{-r x}/r int_0^inf e^{-u} [f(t) e^{r t}] du by Gauss-Laguerre;
       far out, the expansion above */
    fq log_tail(fq x) const
    {
        if (rate * x >= 80 && alpha * x >= 45) return log_tail_far(x);
        const Laguerre& G = laguerre();
        fq s = 0;
        for (int i = 0; i < GLAG; ++i) {
            fq t = x + G.t[i] / rate;
            s += G.w[i] * expq(log_f(t) + rate * t);
        }
        return logq(s) - rate * x - logq(rate);
    }
    /* p+ from the paper's 2F1 closed form (series after the Pfaff transformation) */
    static fq log_mass(fq lam, fq alpha, fq beta)
    {
        const fq w = (1 + beta / alpha) / 2;
        fq term = 1, F = 1;
        for (int n = 0; n < 200000; ++n) {
            term *= (1 - lam + n) * (lam + n) / ((lam + 1 + n) * (n + 1)) * w;
            F += term;
            if (fabsq(term) <= 1e-36Q * fabsq(F)) break;
        }
        return (lam - 1) * M_LN2q + lam * logq(1 + beta / alpha) + lgammaq(lam + 0.5Q) + logq(F) -
               0.5Q * logq(M_PIq) - lgammaq(lam + 1);
    }

    /* Taylor coefficients of (Q, P) about v0 from Q[0], P[0], with R(alpha Q0)
       from the Bessel solution */
    void vstep(VNode& n) const
    {
        fq R[TM + 1], PP[TM + 1], RPP[TM + 1], RRm[TM + 1], PRR[TM + 1], RP[TM + 1], D[TM + 1];
        fq L;
        bes.eval(alpha * n.Q[0], &R[0], &L);
        for (int k = 0; k < TM; ++k) {
            fq pp = 0, rr = 0, rp = 0;
            for (int i = 0; i <= k; ++i) {
                pp += n.P[i] * n.P[k - i];
                rr += R[i] * R[k - i];
                rp += R[i] * n.P[k - i];
            }
            PP[k] = pp;
            RRm[k] = rr - (k == 0 ? 1 : 0);
            RP[k] = rp;
            fq rpp = 0, prr = 0, qd = 0;
            for (int i = 0; i <= k; ++i) {
                rpp += R[i] * PP[k - i];
                prr += n.P[i] * RRm[k - i];
            }
            for (int i = 1; i <= k; ++i) qd += n.Q[i] * D[k - i];
            RPP[k] = rpp;
            PRR[k] = prr;
            D[k] = (RP[k] - qd) / n.Q[0];                      /* R P / Q */
            n.Q[k + 1] = n.P[k] / (k + 1);
            n.P[k + 1] = (-rate * n.P[k] + alpha * RPP[k] - beta * PP[k]) / (k + 1);
            R[k + 1] = (alpha * PRR[k] + (2 * nu - 1) * D[k]) / (k + 1);
        }
    }
    /* Taylor steps from (v, Q, P) to v1 (steps also within |v|/3 of the
       current point, the distance to the origin's singularity) */
    bool leg(fq v, fq Q, fq P, fq v1, std::vector<VNode>& out) const
    {
        const fq dir = v1 > v ? 1 : -1;
        for (int guard = 0; guard < 20000; ++guard) {
            VNode n;
            n.v0 = v;
            n.Q[0] = Q;
            n.P[0] = P;
            vstep(n);
            fq scale = fabsq(n.Q[0]) + fabsq(n.P[0]) * 1e-3Q + 1e-300Q;
            fq h = fminq(0.25Q + 0.05Q * fabsq(v), fabsq(v) / 3);
            for (int k = TM - 1; k <= TM; ++k) {
                if (n.Q[k] == 0) continue;
                fq hk = powq(1e-36Q * scale / fabsq(n.Q[k]), 1.0Q / k);
                if (hk < h) h = hk;
            }
            const bool last = fabsq(v1 - v) <= h;
            if (last) h = fabsq(v1 - v);
            n.h = dir * h;
            out.push_back(n);
            Q = horner(n.Q, n.h);
            P = horner(n.P, n.h);
            v += n.h;
            if (last) return true;
        }
        return false;
    }
    static fq leg_eval(const std::vector<VNode>& nd, fq v)
    {
        size_t lo = 0, hi = nd.size() - 1;
        const bool up = nd.front().h > 0;
        while (lo < hi) {
            size_t mid = (lo + hi) / 2;
            fq a = nd[mid].v0, b = nd[mid].v0 + nd[mid].h;
            fq lo_v = up ? a : b, hi_v = up ? b : a;
            if (v < lo_v) {
                if (up) hi = mid; else lo = mid + 1;
            } else if (v > hi_v) {
                if (up) lo = mid + 1; else hi = mid;
            } else {
                lo = hi = mid;
            }
        }
        return horner(nd[lo].Q, v - nd[lo].v0);
    }
    /* Newton on the central form int_0^x f = p (1 - e^{-r v}) */
    fq solve_central(fq v) const
    {
        const fq target = -expq(log_p) * expm1q(-rate * v);
        fq x = slope0 * v;
        for (int it = 0; it < 60; ++it) {
            fq dx = (central_mass(x) - target) / expq(log_f(x));
            fq xn = x - dx;
            if (!(xn > 0)) xn = x / 2;
            if (fabsq(xn - x) <= 1e-33Q * xn) return xn;
            x = xn;
        }
        return x;
    }
    /* Newton on log(1 - F(x)) = log p - r v (r x >= 24) */
    fq solve_tail(fq v, fq x0) const
    {
        const fq target = log_p - rate * v;
        fq x = x0;
        for (int it = 0; it < 60; ++it) {
            fq lt = log_tail(x);
            fq xn = x + (lt - target) * expq(lt - log_f(x));
            if (fabsq(xn - x) <= 1e-33Q * xn) return xn;
            x = xn;
        }
        return x;
    }

    fq eval(fq v) const override
    {
        if (v <= v_min) return v * (slope0 + q2 * v);
        if (v <= v_s) return leg_eval(zero, v);
        if (v <= v_match) return leg_eval(fwd, v);
        if (v <= v_a) return leg_eval(bwd, v);
        return solve_tail(v, far(v));
    }

    bool build(fq lam, fq alpha_, fq beta_, char* err, int errlen)
    {
        lambda = lam;
        nu = lam - 0.5Q;
        alpha = alpha_;
        beta = beta_;
        rate = alpha - beta;
        /* |x|^(2 lambda - 1) at 0 (the z^(2 nu) series of K_nu); analytic when
           2 lambda is an integer */
        rho = fmodq(2 * lam, 1) != 0 ? 2 * lam - 1 : 0;
        if (!bes.build(nu, err, errlen)) return false;
        logA = lam * logq((alpha - beta) * (alpha + beta)) - nu * logq(2 * alpha) - 0.5Q * logq(M_PIq) - lgammaq(lam);
        log_f0 = logA - nu * logq(alpha) + bes.L0;
        log_p = log_mass(lam, alpha, beta);
        slope0 = expq(log_p - log_f0) * rate;
        q2 = (-rate * slope0 - beta * slope0 * slope0) / 2;
        /* the large-v form */
        const fq e1 = (4 * nu * nu - 1) / (8 * alpha);
        const fq e2 = (4 * nu * nu - 1) * (4 * nu * nu - 9) / (128 * alpha * alpha);
        const fq s1 = (lam - 1) / rate + e1;
        const fq s2 = (lam - 1) * (lam - 2) / (rate * rate) + e1 * (lam - 2) / rate + e2;
        c0 = (logA + 0.5Q * logq(M_PIq / (2 * alpha)) - logq(rate) - log_p) / rate;
        clog = (lam - 1) / rate;
        c1 = s1 / rate;
        c2 = (s2 - s1 * s1 / 2) / rate;
        /* the masses against quadrature of f: int_0^{x1} by halving panels, the
           tail by Gauss-Laguerre */
        {
            const fq x1 = 24 / rate;
            const fq q = central_mass(x1) + expq(log_tail(x1));
            if (!(fabsq(q / expq(log_p) - 1) < 1e-28Q)) {
                snprintf(err, errlen, "variance-gamma mass: 2F1 form and quadrature differ by %.3e",
                         (double)fabsq(q / expq(log_p) - 1));
                return false;
            }
        }
        v_s = fminq(0.125Q, 0.125Q / rate);
        v_match = 20 / rate;
        fq va = 40 / rate;
        for (int it = 0; it < 100 && rate * far(va) < 30; ++it) va *= 1.25Q;
        v_a = va;
        v_min = fminq(1e-17Q, powq(10, -34 / (2 * lam - 1)));
        const fq Qs = solve_central(v_s);
        const fq Ps = expq(log_p + logq(rate) - rate * v_s - log_f(Qs));
        const fq Qa = solve_tail(v_a, far(v_a));
        if (!(rate * Qa >= 24)) {
            snprintf(err, errlen, "variance-gamma anchor too close to the centre");
            return false;
        }
        const fq Pa = expq(log_p + logq(rate) - rate * v_a - log_f(Qa));
        if (!leg(v_min, v_min * (slope0 + q2 * v_min), slope0 + 2 * q2 * v_min, v_s, zero) ||
            !leg(v_s, Qs, Ps, v_match, fwd) || !leg(v_a, Qa, Pa, v_match, bwd)) {
            snprintf(err, errlen, "the ODE integration exceeded its step budget");
            return false;
        }
        const VNode& f = fwd.back();
        const VNode& b = bwd.back();
        const fq qf = horner(f.Q, f.h), qb = horner(b.Q, b.h);
        const fq pf = horner(f.P, f.h), pb = horner(b.P, b.h);
        const fq mis = fabsq(qf / qb - 1) + fabsq(pf / pb - 1);
        if (!(mis < 1e-19Q)) {
            snprintf(err, errlen, "legs disagree at v=%g by %.3e", (double)v_match, (double)mis);
            return false;
        }
        /* the leg from the origin's series must meet the direct solve at v_s */
        const VNode& z = zero.back();
        const fq mz = fabsq(horner(z.Q, z.h) / Qs - 1) + fabsq(horner(z.P, z.h) / Ps - 1);
        if (!(mz < 1e-19Q)) {
            snprintf(err, errlen, "the leg from the origin misses the direct solve at v=%g by %.3e", (double)v_s,
                     (double)mz);
            return false;
        }
        return true;
    }
};

bool check_vg_params(double lambda, double alpha, double beta)
{
    return std::isfinite(lambda) && std::isfinite(alpha) && std::isfinite(beta) && lambda >= 1 &&
           lambda <= VG_LAMBDA_MAX && alpha > std::fabs(beta);
}

}  // namespace

int build_hyperbolic_table(double alpha, double beta, double delta, HostHypTable* out, char* err, int errlen)
{
    memset(out, 0, sizeof *out);
    if (!check_params(alpha, beta, delta)) return fail(err, errlen, "need |beta| < alpha and delta > 0, all finite");
    HypTableHeader& H = out->hdr;
    H.alpha = alpha;
    H.beta = beta;
    H.delta = delta;
    const Side right = make_side(alpha, beta, delta);
    const Side left = make_side(alpha, -(fq)beta, delta);
    H.log_p_plus = (double)right.log_p;
    H.log_p_minus = (double)left.log_p;
    SideSolution rs, ls;
    if (!solve_side(right, &rs, err, errlen) || !solve_side(left, &ls, err, errlen)) return -1;
    std::vector<double> coef;
    if (!fit_set(rs, ls, CellSpec{HYP_DEGREE, 2e-17Q}, &H.right, &H.left, coef, err, errlen)) return -1;
    if (!fit_set(rs, ls, CellSpec{HYP_DEGREE_F32, 1e-10Q}, &H.right32, &H.left32, coef, err, errlen)) return -1;
    out->ncoef = coef.size();
    out->coef = (double*)malloc(out->ncoef * sizeof(double));
    if (!out->coef) return fail(err, errlen, "out of memory");
    memcpy(out->coef, coef.data(), out->ncoef * sizeof(double));
    return 0;
}

int build_vg_table(double lambda, double alpha, double beta, HostHypTable* out, char* err, int errlen)
{
    memset(out, 0, sizeof *out);
    if (!check_vg_params(lambda, alpha, beta))
        return fail(err, errlen, "need lambda in [1, 8] and |beta| < alpha, all finite");
    HypTableHeader& H = out->hdr;
    H.alpha = alpha;
    H.beta = beta;
    H.delta = lambda;
    std::vector<double> coef;
    if (lambda == std::floor(lambda)) {
        /* integer lambda: each side solved directly from its closed form */
        const int n = (int)lambda - 1;
        const VGSide right(n, alpha, beta), left(n, alpha, -(fq)beta);
        H.log_p_plus = (double)right.log_p;
        H.log_p_minus = (double)left.log_p;
        if (!fit_set(right, left, CellSpec{HYP_DEGREE, 2e-17Q}, &H.right, &H.left, coef, err, errlen)) return -1;
        if (!fit_set(right, left, CellSpec{HYP_DEGREE_F32, 1e-10Q}, &H.right32, &H.left32, coef, err, errlen))
            return -1;
    } else {
        /* real lambda: the recycling ODE */
        VGRealSide right, left;
        if (!right.build(lambda, alpha, beta, err, errlen) || !left.build(lambda, alpha, -(fq)beta, err, errlen))
            return -1;
        H.log_p_plus = (double)right.log_p;
        H.log_p_minus = (double)left.log_p;
        if (!fit_set(right, left, CellSpec{HYP_DEGREE, 2e-17Q}, &H.right, &H.left, coef, err, errlen)) return -1;
        if (!fit_set(right, left, CellSpec{HYP_DEGREE_F32, 1e-10Q}, &H.right32, &H.left32, coef, err, errlen))
            return -1;
    }
    out->ncoef = coef.size();
    out->coef = (double*)malloc(out->ncoef * sizeof(double));
    if (!out->coef) return fail(err, errlen, "out of memory");
    memcpy(out->coef, coef.data(), out->ncoef * sizeof(double));
    return 0;
}

void free_hyperbolic_table(HostHypTable* t)
{
    if (t && t->coef) {
        free(t->coef);
        t->coef = nullptr;
    }
}

}  // namespace qm

/* Host copy of a table (include/qm_debug.h). */
extern "C" int qm_debug_hyperbolic_table(double alpha, double beta, double delta, void* header_out, double* coef_out,
                                         int coef_cap)
{
    qm::HostHypTable t;
    char err[256];
    if (qm::build_hyperbolic_table(alpha, beta, delta, &t, err, sizeof err) != 0) {
        fprintf(stderr, "qm_debug_hyperbolic_table: %s\n", err);
        return -1;
    }
    int need = (int)t.ncoef;
    if (header_out) memcpy(header_out, &t.hdr, sizeof t.hdr);
    if (coef_out && coef_cap >= need && need > 0) memcpy(coef_out, t.coef, sizeof(double) * need);
    qm::free_hyperbolic_table(&t);
    return need;
}

/* Dense ODE solution (include/qm_debug.h). */
extern "C" int qm_debug_hyperbolic_dense(double alpha, double beta, double delta, const double* v, double* q, int n)
{
    using namespace qm;
    if (!check_params(alpha, beta, delta) || n < 0) return -1;
    char err[256];
    const Side right = make_side(alpha, beta, delta);
    const Side left = make_side(alpha, -(fq)beta, delta);
    SideSolution rs, ls;
    if (!solve_side(right, &rs, err, sizeof err) || !solve_side(left, &ls, err, sizeof err)) {
        fprintf(stderr, "qm_debug_hyperbolic_dense: %s\n", err);
        return -1;
    }
    for (int i = 0; i < n; ++i) {
        fq x = v[i];
        const SideSolution& ss = x >= 0 ? rs : ls;
        fq a = fabsq(x);
        if (!(a <= 1e12Q)) return -1;
        fq Q = a == 0 ? (fq)0 : ss.eval(a);
        q[i] = (double)(x >= 0 ? Q : -Q);
    }
    return 0;
}

/* Host copy of a variance-gamma table (include/qm_debug.h). */
extern "C" int qm_debug_vg_table(double lambda, double alpha, double beta, void* header_out, double* coef_out,
                                 int coef_cap)
{
    qm::HostHypTable t;
    char err[256];
    if (qm::build_vg_table(lambda, alpha, beta, &t, err, sizeof err) != 0) {
        fprintf(stderr, "qm_debug_vg_table: %s\n", err);
        return -1;
    }
    int need = (int)t.ncoef;
    if (header_out) memcpy(header_out, &t.hdr, sizeof t.hdr);
    if (coef_out && coef_cap >= need && need > 0) memcpy(coef_out, t.coef, sizeof(double) * need);
    qm::free_hyperbolic_table(&t);
    return need;
}

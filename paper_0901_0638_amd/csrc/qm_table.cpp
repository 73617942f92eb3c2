/*
 * qm_table.cpp -- host builder of the normal -> Student t tables.
 *
 * The map Q(z) = F_nu^{-1}(Phi(z)) solves the recycling ODE with a Gaussian
 * background (Section 3.1):
 *
 *     (nu + Q^2) (Q'' + z Q') = (nu + 1) Q Q'^2,   Q(0) = 0, Q'(0) = gamma,
 *     gamma = sqrt(nu/2) Gamma(nu/2) / Gamma((nu+1)/2).
 *
 * Following the paper's method (solve the RODE numerically, then build a fast
 * approximation, Sections 3.6 and 9), the builder integrates it by the Taylor
 * series method -- the central expansion of Section 3.2 generalised to an
 * arbitrary expansion point z0: substituting Q = sum a_k (z - z0)^k and
 * matching powers gives a_{k+2} from a_0..a_{k+1} (see taylor_step) -- in
 * __float128.  Integrating outwards is ill-conditioned in the tail: the ODE
 * also admits F^{-1}(a + Phi(z)), and a perturbation a grows relative to the
 * solution like 1/(1 - Phi(z)).  So the solution is built from both ends:
 *
 *   forward  from the centre conditions to z_m = 4,
 *   backward from z_far = 10.5 down to z_m, starting from the tail
 *            condition: Q(z_far) solves 1 - F_nu(Q) = 1 - Phi(z_far) with the
 *            Student tail written as a convergent hypergeometric series
 *            (DLMF 8.17.8), Q'(z_far) = phi(z_far) / f_nu(Q) (the centre/tail
 *            boundary data of Sections 3.1 and 3.3),
 *
 * and the two legs must agree at z_m (checked).  The device table then holds,
 * for y = z^2 in [0, 100], cells of width h in y with the Chebyshev
 * interpolant of R(y) = Q(z)/z (an even function of z, like the paper's
 * series in y = z^2, Section 3.5), stored as monomial coefficients in
 * d = y - y_centre.  For nu > 1e5 the map is within 1e-19 of the
 * Cornish-Fisher series of Section 3.4 (A&S 26.7.5), used directly.
 */
#include <quadmath.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "qm_table.h"

namespace qm {
namespace {

typedef __float128 fq;

constexpr int TAYLOR_M = 32;        /* Taylor order of the integrator */
constexpr double Z_MATCH = 4.0;     /* forward/backward meeting point */
constexpr double Z_FAR = 10.5;      /* backward anchor */
constexpr double Y_TABLE = 100.0;   /* table covers y = z^2 in [0, Y_TABLE] */
constexpr double NU_CF = 1e5;       /* above: Cornish-Fisher polynomial */

struct Node {
    fq z0, h;                       /* expansion point and the step taken from it (signed) */
    fq a[TAYLOR_M + 1];
};

/*
 * Taylor coefficients of the RODE solution about z0, given a[0] = Q(z0) and
 * a[1] = Q'(z0).  With b_k = (k+1) a_{k+1} (Q'), c_k = (k+2)(k+1) a_{k+2}
 * (Q''), s_k = c_k + z0 b_k + b_{k-1} (Q'' + z Q'), the power d^k of
 * (nu + Q^2) S = (nu + 1) Q Q'^2 is
 *   (nu + a0^2) c_k + (nu + a0^2)(z0 b_k + b_{k-1}) + sum_{i>=1} q2_i s_{k-i}
 *       = (nu + 1) sum_i a_i p2_{k-i},
 * q2 = Q^2 and p2 = Q'^2 as convolutions; it is solved for a_{k+2}.
 */
void taylor_step(fq nu, fq z0, fq* a, int M)
{
    fq b[TAYLOR_M + 2], s[TAYLOR_M + 2], q2[TAYLOR_M + 2], p2[TAYLOR_M + 2];
    const fq lead = nu + a[0] * a[0];
    for (int k = 0; k + 2 <= M; ++k) {
        b[k] = (fq)(k + 1) * a[k + 1];
        q2[k] = 0;
        for (int i = 0; i <= k; ++i) q2[k] += a[i] * a[k - i];
        p2[k] = 0;
        for (int i = 0; i <= k; ++i) p2[k] += b[i] * b[k - i];
        fq rhs = 0;
        for (int i = 0; i <= k; ++i) rhs += a[i] * p2[k - i];
        rhs *= (nu + 1);
        fq zb = z0 * b[k] + (k > 0 ? b[k - 1] : (fq)0);
        fq acc = lead * zb;
        for (int i = 1; i <= k; ++i) acc += q2[i] * s[k - i];
        fq c = (rhs - acc) / lead;
        a[k + 2] = c / ((fq)(k + 2) * (fq)(k + 1));
        s[k] = c + zb;
    }
}

fq horner_q(const fq* a, int M, fq d)
{
    fq r = a[M];
    for (int k = M - 1; k >= 0; --k) r = r * d + a[k];
    return r;
}

fq horner_qd(const fq* a, int M, fq d)
{
    fq r = (fq)M * a[M];
    for (int k = M - 1; k >= 1; --k) r = r * d + (fq)k * a[k];
    return r;
}

/* Largest |h| with the last two Taylor terms below tol |Q| (and <= hmax). */
fq step_size(const fq* a, int M, fq hmax)
{
    const fq tol = 1e-36Q;
    fq scale = fabsq(a[0]) + fabsq(a[1]) * 1e-3Q + 1e-300Q;
    fq h = hmax;
    for (int k = M - 1; k <= M; ++k) {
        if (a[k] == 0) continue;
        fq hk = powq(tol * scale / fabsq(a[k]), 1.0Q / k);
        if (hk < h) h = hk;
    }
    return h;
}

/* Integrate from (z0, Q, Q') to z1 (either direction), recording nodes. */
void integrate(fq nu, fq z0, fq Q, fq dQ, fq z1, std::vector<Node>& out)
{
    fq dir = z1 > z0 ? 1 : -1;
    fq z = z0;
    for (int guard = 0; guard < 100000; ++guard) {
        Node n;
        n.z0 = z;
        n.a[0] = Q;
        n.a[1] = dQ;
        taylor_step(nu, z, n.a, TAYLOR_M);
        fq h = step_size(n.a, TAYLOR_M, 0.25Q);
        bool last = false;
        if (fabsq(z1 - z) <= h) { h = fabsq(z1 - z); last = true; }
        n.h = dir * h;
        out.push_back(n);
        Q = horner_q(n.a, TAYLOR_M, n.h);
        dQ = horner_qd(n.a, TAYLOR_M, n.h);
        z += n.h;
        if (last) break;
    }
}

fq lgamma_q(fq x) { return lgammaq(x); }

/*
 * Student upper tail T(t) = 1 - F_nu(t), t > 0, from DLMF 8.17.8:
 *   I_x(a, b) = x^a (1-x)^b / (a B(a,b)) 2F1(a+b, 1; a+1; x),
 * a = nu/2, b = 1/2, x = nu/(nu + t^2), T = I_x(a,b)/2.  Returns log T.
 */
fq log_student_upper(fq nu, fq t, fq lbeta)
{
    fq t2 = t * t;
    fq x = nu / (nu + t2), omx = t2 / (nu + t2);
    fq a = nu / 2, c = a + 1, ab = a + 0.5Q;
    fq term = 1, sum = 1;
    for (long n = 0; n < 50000000; ++n) {
        term *= (ab + n) / (c + n) * x;
        sum += term;
        if (term < 1e-36Q * sum) break;
    }
    return a * logq(x) + 0.5Q * logq(omx) - logq(nu) - lbeta + logq(sum);
}

/* Student density f_nu(t) (Section 3.1), log form. */
fq log_student_pdf(fq nu, fq t, fq lbeta)
{
    return -0.5Q * logq(nu) - lbeta - (nu + 1) / 2 * log1pq(t * t / nu);
}

/* Q(z_far): solve log T(t) = log q by Newton from the tail formula guess. */
fq anchor_value(fq nu, fq zf, fq lbeta, fq logq_target)
{
    /* guess: t = sqrt(nu) w^{-1/nu}, w = q nu sqrt(pi) G(nu/2)/G((nu+1)/2) (Section 3.3) */
    fq logK = logq(nu) + 0.5Q * logq(M_PIq) + lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2);
    fq t = sqrtq(nu) * expq(-(logK + logq_target) / nu);
    if (!(t > zf * 0.5Q)) t = zf;
    for (int it = 0; it < 200; ++it) {
        fq g = log_student_upper(nu, t, lbeta) - logq_target;
        /* d log T / dt = -f(t) / T(t) */
        fq dg = -expq(log_student_pdf(nu, t, lbeta) - log_student_upper(nu, t, lbeta));
        fq tn = t - g / dg;
        if (tn <= 0) tn = t * 0.5Q;
        if (fabsq(tn - t) <= 1e-32Q * t) { t = tn; break; }
        t = tn;
    }
    return t;
}

/* Dense output Q(z), 0 <= z <= Z_FAR, from the recorded nodes. */
struct Solution {
    std::vector<Node> fwd, bwd;
    fq eval(fq z) const
    {
        const std::vector<Node>& v = (z <= (fq)Z_MATCH) ? fwd : bwd;
        /* node whose step covers z */
        size_t best = 0;
        fq bd = 1e300Q;
        for (size_t i = 0; i < v.size(); ++i) {
            fq lo = v[i].h > 0 ? v[i].z0 : v[i].z0 + v[i].h;
            fq hi = v[i].h > 0 ? v[i].z0 + v[i].h : v[i].z0;
            fq dist = z < lo ? lo - z : (z > hi ? z - hi : (fq)0);
            if (dist < bd) { bd = dist; best = i; if (dist == 0) break; }
        }
        return horner_q(v[best].a, TAYLOR_M, z - v[best].z0);
    }
};

/* Chebyshev interpolant of f on [y0 - hw, y0 + hw] as monomials in d = y - y0. */
void cheb_to_monomial(const fq* fv, int K, fq hw, fq* mono)
{
    /* values at nodes x_i = cos(pi (i + 1/2)/(K+1)) -> Chebyshev coefficients */
    const int N = K + 1;
    fq ck[64];
    for (int j = 0; j < N; ++j) {
        fq s = 0;
        for (int i = 0; i < N; ++i) s += fv[i] * cosq(M_PIq * j * (i + 0.5Q) / N);
        ck[j] = s * 2 / N;
    }
    ck[0] /= 2;
    /* sum_j ck_j T_j(x) -> monomials in x via the three-term recurrence */
    fq Tprev[64], Tcur[64], Tnext[64];
    for (int i = 0; i < N; ++i) { mono[i] = 0; Tprev[i] = 0; Tcur[i] = 0; }
    Tprev[0] = 1;             /* T0 */
    Tcur[1] = 1;              /* T1 */
    for (int i = 0; i < N; ++i) mono[i] += ck[0] * Tprev[i];
    if (N > 1) for (int i = 0; i < N; ++i) mono[i] += ck[1] * Tcur[i];
    for (int j = 2; j < N; ++j) {
        for (int i = 0; i < N; ++i) Tnext[i] = -Tprev[i] + (i > 0 ? 2 * Tcur[i - 1] : (fq)0);
        for (int i = 0; i < N; ++i) mono[i] += ck[j] * Tnext[i];
        memcpy(Tprev, Tcur, sizeof(fq) * N);
        memcpy(Tcur, Tnext, sizeof(fq) * N);
    }
    /* x = d / hw */
    fq sc = 1;
    for (int i = 0; i < N; ++i) { mono[i] /= sc; sc *= hw; }
}

int fail(char* err, int errlen, const char* msg)
{
    snprintf(err, errlen, "%s", msg);
    return -1;
}

}  // namespace

int build_student_table(double nu_d, HostTTable* out, char* err, int errlen)
{
    memset(out, 0, sizeof *out);
    if (!(nu_d >= 0.5)) return fail(err, errlen, "nu must be >= 0.5");
    TTableHeader& H = out->hdr;
    H.nu = nu_d;
    if (std::isinf(nu_d)) {
        H.identity = 1;
        H.ncell = 0;
        H.degree = 0;
        H.stride = 0;
        H.h = 1;
        H.inv_h = 1;
        H.y_max = 0;
        return 0;
    }
    const fq nu = nu_d;
    const fq lbeta = lgamma_q(nu / 2) + lgamma_q(0.5Q) - lgamma_q(nu / 2 + 0.5Q);
    H.log_K = (double)(logq(nu) + 0.5Q * logq(M_PIq) + lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2));
    /* two-term tail of Section 3.5: t = sqrt(nu) w^{-1/nu} (1 - (nu+1)/(2(nu+2)) w^{2/nu}) */
    H.tail_a[0] = -(double)((nu + 1) / (2 * (nu + 2)));

    const int K = 15;                     /* polynomial degree per cell */
    H.degree = K;
    H.stride = K + 1;

    if (nu_d > NU_CF) {
        /* Section 3.4 (A&S 26.7.5): t = z (1 + (y+1)/(4n) + (5y^2+16y+3)/(96n^2)
           + (3y^3+19y^2+17y-15)/(384n^3) + (79y^4+776y^3+1482y^2-1920y-945)/(92160n^4)),
           one cell whose polynomial in d = y (y_centre = 0) covers all y. */
        H.identity = 0;
        H.ncell = 1;
        H.h = 1e300;
        H.inv_h = 0;
        H.y_max = 1e300;
        H.centre_offset = 0;
        out->coef = (double*)calloc(H.stride, sizeof(double));
        if (!out->coef) return fail(err, errlen, "out of memory");
        fq n = nu, c[5] = {0, 0, 0, 0, 0};
        c[0] = 1 + 1 / (4 * n) + 3 / (96 * n * n) - 15 / (384 * n * n * n) - 945 / (92160 * n * n * n * n);
        c[1] = 1 / (4 * n) + 16 / (96 * n * n) + 17 / (384 * n * n * n) - 1920 / (92160 * n * n * n * n);
        c[2] = 5 / (96 * n * n) + 19 / (384 * n * n * n) + 1482 / (92160 * n * n * n * n);
        c[3] = 3 / (384 * n * n * n) + 776 / (92160 * n * n * n * n);
        c[4] = 79 / (92160 * n * n * n * n);
        /* stored highest power first, degree K */
        for (int k = 0; k <= 4; ++k) out->coef[K - k] = (double)c[k];
        out->max_rel_err = 0;
        return 0;
    }

    /* --- the two legs of the RODE solution ------------------------------- */
    Solution sol;
    const fq gamma = sqrtq(nu / 2) * expq(lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2));
    integrate(nu, 0, 0, gamma, Z_MATCH, sol.fwd);
    const fq zf = Z_FAR;
    const fq logq_far = logq(erfcq(zf / sqrtq(2)) / 2);
    const fq Qf = anchor_value(nu, zf, lbeta, logq_far);
    const fq phi_far = expq(-zf * zf / 2) / sqrtq(2 * M_PIq);
    const fq dQf = phi_far / expq(log_student_pdf(nu, Qf, lbeta));
    integrate(nu, zf, Qf, dQf, Z_MATCH, sol.bwd);
    /* the legs meet at z_m: value and slope must agree */
    {
        const Node& f = sol.fwd.back();
        const Node& b = sol.bwd.back();
        fq qf = horner_q(f.a, TAYLOR_M, f.h), qb = horner_q(b.a, TAYLOR_M, b.h);
        fq df = horner_qd(f.a, TAYLOR_M, f.h), db = horner_qd(b.a, TAYLOR_M, b.h);
        fq mis = fabsq(qf / qb - 1) + fabsq(df / db - 1);
        if (!(mis < 1e-22Q)) {
            char buf[128];
            snprintf(buf, sizeof buf, "forward/backward legs disagree at z=%g by %.3e", Z_MATCH, (double)mis);
            return fail(err, errlen, buf);
        }
    }

    /* --- cells: the widest h (power of 2) whose Chebyshev interpolants have
       truncation error < 2e-17 (checked with the exact coefficients); the
       error after rounding the coefficients to FP64 (about an ulp of R) is
       measured as well and reported ------------------------------------- */
    const fq tol = 2e-17Q;
    for (double h = 8.0; h >= 1.0 / 64; h /= 2) {
        int ncell = (int)std::ceil(Y_TABLE / h);
        if (ncell > 480) break;   /* 480 rows of 17 doubles fit the 64 KB of LDS a launch may use */
        std::vector<double> coef((size_t)ncell * H.stride, 0.0);
        fq worst = 0;
        bool ok = true;
        for (int j = 0; j < ncell && ok; ++j) {
            fq yc = (j + 0.5Q) * h, hw = 0.5Q * h;
            fq fv[64], mono[64];
            for (int i = 0; i <= K; ++i) {
                fq x = cosq(M_PIq * (i + 0.5Q) / (K + 1));
                fq y = yc + hw * x;
                fq z = sqrtq(y);
                fv[i] = z > 0 ? sol.eval(z) / z : gamma;
            }
            cheb_to_monomial(fv, K, hw, mono);
            for (int k = 0; k <= K; ++k) coef[(size_t)j * H.stride + (K - k)] = (double)mono[k];
            for (int t = 0; t <= 4 * K; ++t) {
                fq d = -hw + h * (fq)t / (4 * K);
                fq y = yc + d;
                fq z = sqrtq(y);
                fq ref = z > 0 ? sol.eval(z) / z : gamma;
                fq pe = 0, pr = 0;
                for (int k = K; k >= 0; --k) pe = pe * d + mono[k];
                for (int k = 0; k <= K; ++k) pr = pr * d + (fq)coef[(size_t)j * H.stride + k];
                fq et = fabsq(pe / ref - 1), er = fabsq(pr / ref - 1);
                if (er > worst) worst = er;
#ifdef QM_TABLE_VERBOSE
                if (et > tol) fprintf(stderr, "h %g cell %d y %g trunc err %.3e\n", h, j, (double)y, (double)et);
#endif
                if (et > tol) { ok = false; break; }
            }
        }
        if (!ok) continue;
        H.identity = 0;
        H.ncell = ncell;
        H.h = h;
        H.inv_h = 1.0 / h;
        H.y_max = ncell * h;
        H.centre_offset = 0.5 * h;
        out->coef = (double*)malloc(coef.size() * sizeof(double));
        if (!out->coef) return fail(err, errlen, "out of memory");
        memcpy(out->coef, coef.data(), coef.size() * sizeof(double));
        out->max_rel_err = (double)worst;
        return 0;
    }
    return fail(err, errlen, "no cell width met the accuracy target");
}

void free_student_table(HostTTable* t)
{
    if (t && t->coef) {
        free(t->coef);
        t->coef = nullptr;
    }
}

}  // namespace qm

/* Dense RODE solution (include/qm_debug.h). */
extern "C" int qm_debug_student_dense(double nu_d, const double* z, double* q, int n)
{
    using namespace qm;
    if (!(nu_d >= 0.5) || nu_d > NU_CF) return -1;
    const fq nu = nu_d;
    const fq lbeta = lgamma_q(nu / 2) + lgamma_q(0.5Q) - lgamma_q(nu / 2 + 0.5Q);
    Solution sol;
    const fq gamma = sqrtq(nu / 2) * expq(lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2));
    integrate(nu, 0, 0, gamma, Z_MATCH, sol.fwd);
    const fq zf = Z_FAR;
    const fq logq_far = logq(erfcq(zf / sqrtq(2)) / 2);
    const fq Qf = anchor_value(nu, zf, lbeta, logq_far);
    const fq dQf = expq(-zf * zf / 2) / sqrtq(2 * M_PIq) / expq(log_student_pdf(nu, Qf, lbeta));
    integrate(nu, zf, Qf, dQf, Z_MATCH, sol.bwd);
    for (int i = 0; i < n; ++i) q[i] = (double)sol.eval(fabsq((fq)z[i])) * (z[i] < 0 ? -1 : 1);
    return 0;
}

/* Host copy of a table (include/qm_debug.h). */
extern "C" int qm_debug_student_table(double nu, void* header_out, double* coef_out, int coef_cap,
                                      double* max_rel_err)
{
    qm::HostTTable t;
    char err[256];
    if (qm::build_student_table(nu, &t, err, sizeof err) != 0) return -1;
    int need = t.hdr.ncell * t.hdr.stride;
    if (header_out) memcpy(header_out, &t.hdr, sizeof t.hdr);
    if (coef_out && coef_cap >= need && need > 0) memcpy(coef_out, t.coef, sizeof(double) * need);
    if (max_rel_err) *max_rel_err = t.max_rel_err;
    qm::free_student_table(&t);
    return need;
}

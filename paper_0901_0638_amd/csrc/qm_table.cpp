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
 *   backward from z_far (10.5, or past the last cell) down to z_m, from the tail
 *            condition: Q(z_far) solves 1 - F_nu(Q) = 1 - Phi(z_far) with the
 *            Student tail written as a convergent hypergeometric series
 *            (DLMF 8.17.8), Q'(z_far) = phi(z_far) / f_nu(Q) (the centre/tail
 *            boundary data of Sections 3.1 and 3.3),
 *
 * and the two legs must agree at z_m (checked).  The device table then holds
 * cells of width h in y = z^2 with the Chebyshev interpolant of
 * R(y) = Q(z)/z (an even function of z, like the paper's series in y = z^2,
 * Section 3.5), stored as monomial coefficients in d = y - y_centre, twice:
 * for FP64 outputs (degree 7 where at most 200 cells cover y <= 100, else
 * degree 15 on wider cells) and for FP32 outputs (degree 7, to 1e-10).  The cells cover y <= 100 and then as far as the two-term tail
 * formula of Section 3.5 falls short of the same accuracy (it is
 * O(w^{4/nu}), so for large nu it needs very large |z|), but never past
 * |z| = 40, beyond the normal quantile of any positive double.  For
 * nu > 1e5 the map is within 1e-19 of the Cornish-Fisher series of
 * Section 3.4 (A&S 26.7.5), used directly.
 */
#include <quadmath.h>

#include <cfloat>
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
constexpr double Z_FAR = 10.5;      /* backward anchor, at least */
constexpr double Y_LDS = 100.0;     /* cells staged in LDS cover y = z^2 in [0, Y_LDS] at least */
constexpr double Z_TAIL0 = 10.0;    /* the tail formula is never used below |z| = Z_TAIL0 */
constexpr double Z_CAP = 40.0;      /* ... and always beyond Z_CAP (past every normal
                                       quantile of a positive double, |z| <= 38.5) */
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

/* Dense output Q(z), 0 <= z <= z_far, from the recorded nodes. */
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

/*
 * The two legs of the RODE solution on [0, z_far]: forward from the centre
 * conditions Q(0) = 0, Q'(0) = gamma to z_m, backward from the tail
 * condition at z_far; they must agree in value and slope at z_m.
 */
bool solve_rode(fq nu, fq lbeta, fq gamma, fq z_far, Solution& sol, char* err, int errlen)
{
    integrate(nu, 0, 0, gamma, Z_MATCH, sol.fwd);
    const fq logq_far = logq(erfcq(z_far / sqrtq(2)) / 2);
    const fq Qf = anchor_value(nu, z_far, lbeta, logq_far);
    const fq phi_far = expq(-z_far * z_far / 2) / sqrtq(2 * M_PIq);
    const fq dQf = phi_far / expq(log_student_pdf(nu, Qf, lbeta));
    integrate(nu, z_far, Qf, dQf, Z_MATCH, sol.bwd);
    const Node& f = sol.fwd.back();
    const Node& b = sol.bwd.back();
    fq qf = horner_q(f.a, TAYLOR_M, f.h), qb = horner_q(b.a, TAYLOR_M, b.h);
    fq df = horner_qd(f.a, TAYLOR_M, f.h), db = horner_qd(b.a, TAYLOR_M, b.h);
    fq mis = fabsq(qf / qb - 1) + fabsq(df / db - 1);
    if (!(mis < 1e-22Q)) {
        snprintf(err, errlen, "forward/backward legs disagree at z=%g by %.3e", Z_MATCH, (double)mis);
        return false;
    }
    return true;
}

/*
 * Where the two-term tail of Section 3.5, t = sqrt(nu) w^{-1/nu}
 * (1 + a w^{2/nu}), w = K q(z), is accurate to tol: the smallest z on a
 * grid of 1/2 in [Z_TAIL0, Z_CAP] from which on its relative error against
 * the exact map (the tail-condition solve at z) stays below tol; Z_CAP if
 * none.  The error falls monotonically with z (it is O(w^{4/nu})), so the
 * scan runs down from Z_CAP and stops at the first failure.
 */
fq tail_formula_z(fq nu, fq lbeta, fq logK, fq a, fq tol)
{
    fq z_ok = Z_CAP;
    for (fq z = Z_CAP; z >= (fq)Z_TAIL0; z -= 0.5Q) {
        fq lq = logq(erfcq(z / sqrtq(2)) / 2);
        fq exact = anchor_value(nu, z, lbeta, lq);
        fq lw = logK + lq;
        fq tf = sqrtq(nu) * expq(-lw / nu) * (1 + a * expq(2 * lw / nu));
        if (!(fabsq(tf / exact - 1) <= tol)) break;
        z_ok = z;
    }
    return z_ok;
}

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

/*
 * Cells of degree K for R(y) = Q(z)/z on y in [0, max(y_need, Y_LDS)]: the
 * widest power-of-2 width h <= 8 whose Chebyshev interpolants have
 * truncation error below tol (checked with the exact coefficients on 4K+1
 * points per cell) and whose cells up to Y_LDS number at most max_lds; the
 * error after rounding the coefficients to FP64 is measured as well and
 * recorded.  Appends the rows to `coef` and fills `c`.  Returns false if
 * no width qualifies.
 */
bool fit_cells(const Solution& sol, fq gamma, int K, fq tol, double y_need, int max_lds, std::vector<double>& coef,
               TCells* c)
{
    const int stride = K + 1;
    const double y_top = y_need > Y_LDS ? y_need : Y_LDS;
    for (double h = 8.0; h >= 1.0 / 256; h /= 2) {
        const int nlds = (int)std::ceil(Y_LDS / h);
        if (nlds > max_lds) break;
        const int ncell = (int)std::ceil(y_top / h);
        std::vector<double> rows((size_t)ncell * stride, 0.0);
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
            double* row = &rows[(size_t)j * stride];
            for (int k = 0; k <= K; ++k) row[K - k] = (double)mono[k];
            for (int t = 0; t <= 4 * K; ++t) {
                fq d = -hw + h * (fq)t / (4 * K);
                fq y = yc + d;
                fq z = sqrtq(y);
                fq ref = z > 0 ? sol.eval(z) / z : gamma;
                fq pe = 0, pr = 0;
                for (int k = K; k >= 0; --k) pe = pe * d + mono[k];
                for (int k = 0; k <= K; ++k) pr = pr * d + (fq)row[k];
                fq et = fabsq(pe / ref - 1), er = fabsq(pr / ref - 1);
                if (er > worst) worst = er;
#ifdef QM_TABLE_VERBOSE
                if (et > tol) fprintf(stderr, "K %d h %g cell %d y %g trunc err %.3e\n", K, h, j, (double)y, (double)et);
#endif
                if (et > tol) { ok = false; break; }
            }
        }
        if (!ok) continue;
        c->h = h;
        c->inv_h = 1.0 / h;
        c->y_max = ncell * h;
        c->y_lds = nlds * h;
        c->centre_offset = 0.5 * h;
        c->max_rel_err = (double)worst;
        c->ncell = ncell;
        c->nlds = nlds;
        c->degree = K;
        c->stride = stride;
        c->coef_offset = coef.size();
        coef.insert(coef.end(), rows.begin(), rows.end());
        return true;
    }
    return false;
}

/* nu > NU_CF: one cell whose polynomial in d = y (centre 0) is the series of
   Section 3.4 (A&S 26.7.5), covering every y,
     t = z (1 + (y+1)/(4n) + (5y^2+16y+3)/(96n^2) + (3y^3+19y^2+17y-15)/(384n^3)
            + (79y^4+776y^3+1482y^2-1920y-945)/(92160n^4)). */
void cornish_fisher_cells(fq n, int K, std::vector<double>& coef, TCells* c)
{
    fq a[5];
    a[0] = 1 + 1 / (4 * n) + 3 / (96 * n * n) - 15 / (384 * n * n * n) - 945 / (92160 * n * n * n * n);
    a[1] = 1 / (4 * n) + 16 / (96 * n * n) + 17 / (384 * n * n * n) - 1920 / (92160 * n * n * n * n);
    a[2] = 5 / (96 * n * n) + 19 / (384 * n * n * n) + 1482 / (92160 * n * n * n * n);
    a[3] = 3 / (384 * n * n * n) + 776 / (92160 * n * n * n * n);
    a[4] = 79 / (92160 * n * n * n * n);
    c->h = 1e300;
    c->inv_h = 0;
    c->y_max = 1e300;
    c->y_lds = 1e300;
    c->centre_offset = 0;
    c->max_rel_err = 0;
    c->ncell = 1;
    c->nlds = 1;
    c->degree = K;
    c->stride = K + 1;
    c->coef_offset = coef.size();
    std::vector<double> row(K + 1, 0.0);
    for (int k = 0; k <= 4; ++k) row[K - k] = (double)a[k];   /* highest power first */
    coef.insert(coef.end(), row.begin(), row.end());
}

}  // namespace

int build_student_table(double nu_d, HostTTable* out, char* err, int errlen)
{
    memset(out, 0, sizeof *out);
    if (!(nu_d >= T_NU_MIN)) return fail(err, errlen, "nu below the smallest tabulated value");
    TTableHeader& H = out->hdr;
    H.nu = nu_d;
    if (std::isinf(nu_d)) {
        H.identity = 1;
        return 0;
    }
    const fq nu = nu_d;
    const fq lbeta = lgamma_q(nu / 2) + lgamma_q(0.5Q) - lgamma_q(nu / 2 + 0.5Q);
    H.log_K = (double)(logq(nu) + 0.5Q * logq(M_PIq) + lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2));
    /* two-term tail of Section 3.5: t = sqrt(nu) w^{-1/nu} (1 - (nu+1)/(2(nu+2)) w^{2/nu}) */
    H.tail_a[0] = -(double)((nu + 1) / (2 * (nu + 2)));

    std::vector<double> coef;
    if (nu_d > NU_CF) {
        cornish_fisher_cells(nu, T_DEGREE_LOW, coef, &H.f64);
        cornish_fisher_cells(nu, T_DEGREE_F32, coef, &H.f32);
    } else {
        /* Tolerances: FP64 outputs, truncation below 2e-17, so the rounded
           coefficients (about an ulp of R) dominate; FP32 outputs, 1e-10.
           The cells reach as far as the tail formula needs to meet the same
           tolerance; those up to Y_LDS are the ones staged in LDS (for FP64,
           degree 7 if at most 200 rows of 10 doubles do, else degree 15 in at
           most 480 rows of 16 doubles, the 64 KB of LDS a launch may use). */
        const fq tol64 = 2e-17Q, tol32 = 1e-10Q;
        /* the formula's truncation error, with its constants exact (their
           rounding to FP64 is part of the device's evaluation error) */
        const fq logK = logq(nu) + 0.5Q * logq(M_PIq) + lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2);
        const fq a = -(nu + 1) / (2 * (nu + 2));
        const fq z64 = tail_formula_z(nu, lbeta, logK, a, tol64);
        const fq z32 = tail_formula_z(nu, lbeta, logK, a, tol32);
        double y64 = (double)(z64 * z64);
        const double y32 = (double)(z32 * z32);
        /* Below nu = 1/2 the device's evaluation of the tail formula is the
           limit, not its truncation: rounding in log w (erfcx, log) reaches t
           multiplied by 1/nu, 2e-15 at nu = 0.3 against a 2e-15 budget.
           There the FP64 cells continue, from global memory, until t passes
           the largest double (the products z R then overflow to +-inf as
           the map does; FP32 outputs overflow long before their cells end). */
        if (nu_d < 0.5) {
            /* the first z (to 0.005) with log t past log(DBL_MAX) + 1; the last
               cell ends at most h later in y, so R = t/z, and its Taylor
               coefficients (about R/(2 nu)^k/k!), stay finite doubles */
            fq zo = (fq)Z_TAIL0;
            for (; zo < (fq)Z_CAP; zo += 0.005Q) {
                const fq lw = logK + logq(erfcq(zo / sqrtq(2)) / 2);
                if (0.5Q * logq(nu) - lw / nu > logq((fq)DBL_MAX) + 1) break;
            }
            if ((double)(zo * zo) > y64) y64 = (double)(zo * zo);
        }
        /* the solution must reach the last cell's upper edge (y rounded up by < 8) */
        fq z_far = sqrtq((fq)(y64 > Y_LDS ? y64 : Y_LDS) + 8) + 0.25Q;
        if (z_far < (fq)Z_FAR) z_far = Z_FAR;
        Solution sol;
        const fq gamma = sqrtq(nu / 2) * expq(lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2));
        if (!solve_rode(nu, lbeta, gamma, z_far, sol, err, errlen)) return -1;
        if (!fit_cells(sol, gamma, T_DEGREE_LOW, tol64, y64, T_LDS_CELLS_LOW, coef, &H.f64) &&
            !fit_cells(sol, gamma, T_DEGREE_HIGH, tol64, y64, 480, coef, &H.f64))
            return fail(err, errlen, "no cell width met the FP64 accuracy target");
        if (!fit_cells(sol, gamma, T_DEGREE_F32, tol32, y32, 720, coef, &H.f32))
            return fail(err, errlen, "no cell width met the FP32 accuracy target");
    }
    out->coef = (double*)malloc(coef.size() * sizeof(double));
    if (!out->coef) return fail(err, errlen, "out of memory");
    memcpy(out->coef, coef.data(), coef.size() * sizeof(double));
    out->ncoef = coef.size();
    return 0;
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
    if (!(nu_d >= T_NU_MIN) || nu_d > NU_CF) return -1;
    fq zmax = 0;
    for (int i = 0; i < n; ++i) {
        fq a = fabsq((fq)z[i]);
        if (!(a <= (fq)Z_CAP)) return -1;
        if (a > zmax) zmax = a;
    }
    const fq nu = nu_d;
    const fq lbeta = lgamma_q(nu / 2) + lgamma_q(0.5Q) - lgamma_q(nu / 2 + 0.5Q);
    const fq gamma = sqrtq(nu / 2) * expq(lgamma_q(nu / 2) - lgamma_q((nu + 1) / 2));
    fq z_far = zmax + 0.5Q;
    if (z_far < (fq)Z_FAR) z_far = Z_FAR;
    Solution sol;
    char err[160];
    if (!solve_rode(nu, lbeta, gamma, z_far, sol, err, sizeof err)) return -1;
    for (int i = 0; i < n; ++i) q[i] = (double)sol.eval(fabsq((fq)z[i])) * (z[i] < 0 ? -1 : 1);
    return 0;
}

/* Host copy of a table (include/qm_debug.h). */
extern "C" int qm_debug_student_table(double nu, void* header_out, double* coef_out, int coef_cap)
{
    qm::HostTTable t;
    char err[256];
    if (qm::build_student_table(nu, &t, err, sizeof err) != 0) return -1;
    int need = (int)t.ncoef;
    if (header_out) memcpy(header_out, &t.hdr, sizeof t.hdr);
    if (coef_out && coef_cap >= need && need > 0) memcpy(coef_out, t.coef, sizeof(double) * need);
    qm::free_student_table(&t);
    return need;
}

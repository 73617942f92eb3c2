/*
 * qm_inputs.c -- seeded synthetic input generators shared by the tests, the
 * oracle checks and the benchmark.  This module holds none of the quantile
 * method's arithmetic: it only turns a counter-based random stream into the
 * arrays the workloads are defined on (uniforms, mixtures, normals,
 * exponentials).
 *
 * Generator: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11): a 4x32-bit counter, a 2x32-bit key,
 * ten rounds of two 32x32->64 multiplies with the published multipliers and
 * a Weyl-sequence key schedule.  Key = (seed, stream); element i of a stream
 * uses counter (i/2 as 64 bits, 0, 0) and takes words (0,1) for even i and
 * words (2,3) for odd i as one 64-bit value, from which the top 53 bits k
 * give the open uniform u = (k + 1/2) 2^-53.  Every element depends only on
 * (seed, stream, i), so any sub-range can be regenerated independently.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <pthread.h>
#include <unistd.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void qmi_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void block(uint64_t seed, uint64_t stream, uint64_t j, uint32_t w[4])
{
    uint32_t ctr[4] = { (uint32_t)j, (uint32_t)(j >> 32), 0u, 0u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)stream };
    qmi_philox4x32_10(ctr, key, w);
}

/* 64 random bits for element i of (seed, stream) */
static uint64_t bits64(uint64_t seed, uint64_t stream, uint64_t i)
{
    uint32_t w[4];
    block(seed, stream, i >> 1, w);
    return (i & 1) ? (((uint64_t)w[3] << 32) | w[2]) : (((uint64_t)w[1] << 32) | w[0]);
}

/* uniform (k + 1/2) 2^-53 with the top 53 bits k, rounded to nearest: a
   tie (to even) for k >= 2^52, and 1.0 for k = 2^53 - 1 */
static double u53(uint64_t bits) { return ((double)(bits >> 11) + 0.5) * 0x1p-53; }

/* open uniform in FP32: (k + 1/2) 2^-23 with the top 23 bits of a word
   (exact: k + 1/2 has at most 24 significant bits, so 0 < u < 1) */
static float u23(uint32_t word) { return ((float)(word >> 9) + 0.5f) * 0x1p-23f; }

/* ---------------------------------------------------------------------- */
typedef struct {
    int kind;
    uint64_t seed, stream;
    size_t begin, end;
    void* out;
    double a, b;  /* kind-specific parameters */
} gjob;

enum {
    G_U53 = 0,        /* open uniform f64 */
    G_U23 = 1,        /* open uniform f32 */
    G_MIX64 = 2,      /* bulk/tail mixture f64 */
    G_MIX32 = 3,      /* bulk/tail mixture f32 */
    G_NORMAL = 4,     /* Box-Muller normals f64 */
    G_EXP = 5,        /* Exp(1) f64 */
};

/*
 * Bulk/tail mixture (per element i): stratum word from stream+1 decides
 * tail with probability a (e.g. 0.1).  Bulk: open uniform from `stream`.
 * Tail: t = exp(log lo + U (log hi - log lo)) with U from stream+2, i.e. t
 * log-uniform in [lo, hi] (lo = b, hi = 1e-2); mirrored to 1 - t with
 * probability 1/2 by a word from stream+3, the subtraction rounded in the
 * output precision.
 */
static double mix_tail(uint64_t seed, uint64_t stream, uint64_t i, double lo, double hi)
{
    double U = u53(bits64(seed, stream + 2, i));
    return exp(log(lo) + U * (log(hi) - log(lo)));
}

static void* gen_run(void* p)
{
    gjob* g = (gjob*)p;
    for (size_t i = g->begin; i < g->end; ++i) {
        switch (g->kind) {
        case G_U53:
            ((double*)g->out)[i] = u53(bits64(g->seed, g->stream, i));
            break;
        case G_U23: {
            uint32_t w[4];
            block(g->seed, g->stream, i >> 2, w);
            ((float*)g->out)[i] = u23(w[i & 3]);
            break;
        }
        case G_MIX64: {
            int tail = u53(bits64(g->seed, g->stream + 1, i)) < g->a;
            double u;
            if (!tail) u = u53(bits64(g->seed, g->stream, i));
            else {
                double t = mix_tail(g->seed, g->stream, i, g->b, 1e-2);
                int mirror = u53(bits64(g->seed, g->stream + 3, i)) < 0.5;
                u = mirror ? 1.0 - t : t;
            }
            ((double*)g->out)[i] = u;
            break;
        }
        case G_MIX32: {
            int tail = u53(bits64(g->seed, g->stream + 1, i)) < g->a;
            float u;
            if (!tail) {
                uint32_t w[4];
                block(g->seed, g->stream, i >> 2, w);
                u = u23(w[i & 3]);
            } else {
                float t = (float)mix_tail(g->seed, g->stream, i, g->b, 1e-2);
                int mirror = u53(bits64(g->seed, g->stream + 3, i)) < 0.5;
                u = mirror ? 1.0f - t : t;
            }
            ((float*)g->out)[i] = u;
            break;
        }
        case G_NORMAL: {
            /* pair j = i/2 from one Philox block: u1 from words (0,1), u2 from
               words (2,3); z_{2j} = r cos(theta), z_{2j+1} = r sin(theta) */
            uint32_t w[4];
            uint64_t j = i >> 1;
            block(g->seed, g->stream, j, w);
            double u1 = u53(((uint64_t)w[1] << 32) | w[0]);
            double u2 = u53(((uint64_t)w[3] << 32) | w[2]);
            double r = sqrt(-2.0 * log(u1));
            double th = 6.283185307179586476925286766559 * u2;
            ((double*)g->out)[i] = (i & 1) ? r * sin(th) : r * cos(th);
            break;
        }
        case G_EXP:
            ((double*)g->out)[i] = -log(u53(bits64(g->seed, g->stream, i)));
            break;
        }
    }
    return NULL;
}

static int gen_parallel(int kind, uint64_t seed, uint64_t stream, void* out, size_t n,
                        double a, double b, int nthreads)
{
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (n < 65536) nthreads = 1;
    pthread_t th[64];
    int joined[64];
    gjob jobs[64];
    size_t per = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        size_t lo = (size_t)t * per, hi = lo + per;
        if (lo > n) lo = n;
        if (hi > n) hi = n;
        jobs[t] = (gjob){ kind, seed, stream, lo, hi, out, a, b };
        joined[t] = 0;
        if (nthreads == 1 || pthread_create(&th[t], NULL, gen_run, &jobs[t]) != 0) {
            gen_run(&jobs[t]);
            continue;
        }
        joined[t] = 1;
    }
    for (int t = 0; t < nthreads; ++t)
        if (joined[t]) pthread_join(th[t], NULL);
    return 0;
}

/* the open-uniform formulas applied to given words (tests of the formulas) */
void qmi_u53_of_bits(const uint64_t* bits, double* out, size_t n)
{ for (size_t i = 0; i < n; ++i) out[i] = u53(bits[i]); }

void qmi_u23_of_words(const uint32_t* words, float* out, size_t n)
{ for (size_t i = 0; i < n; ++i) out[i] = u23(words[i]); }

int qmi_uniform53(uint64_t seed, uint64_t stream, double* out, size_t n, int nthreads)
{ return gen_parallel(G_U53, seed, stream, out, n, 0, 0, nthreads); }

int qmi_uniform23(uint64_t seed, uint64_t stream, float* out, size_t n, int nthreads)
{ return gen_parallel(G_U23, seed, stream, out, n, 0, 0, nthreads); }

int qmi_mixture_f64(uint64_t seed, uint64_t stream, double p_tail, double tail_lo,
                    double* out, size_t n, int nthreads)
{ return gen_parallel(G_MIX64, seed, stream, out, n, p_tail, tail_lo, nthreads); }

int qmi_mixture_f32(uint64_t seed, uint64_t stream, double p_tail, double tail_lo,
                    float* out, size_t n, int nthreads)
{ return gen_parallel(G_MIX32, seed, stream, out, n, p_tail, tail_lo, nthreads); }

int qmi_normals(uint64_t seed, uint64_t stream, double* out, size_t n, int nthreads)
{ return gen_parallel(G_NORMAL, seed, stream, out, n, 0, 0, nthreads); }

int qmi_exponentials(uint64_t seed, uint64_t stream, double* out, size_t n, int nthreads)
{ return gen_parallel(G_EXP, seed, stream, out, n, 0, 0, nthreads); }

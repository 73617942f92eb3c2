/*
 * qm_hyp.hip -- exponential -> hyperbolic recycling kernels (Section 8.1).
 *
 * x = mu + sign(v) Q_side(|v|), Q = a R(a), a = |v|, with R the per-cell
 * polynomial of the side (v >= 0: the right map; v < 0: the mirrored left
 * map) built on the host from the recycling ODE (qm_hyp_table.cpp).  Cells
 * are uniform in t = a / v0 on [0, 1) and eight per octave of t beyond, so
 * the cell index comes from the exponent and the leading mantissa bits of t
 * with no table search.  Each workgroup stages the cells with
 * a < v_lds (64 / rate and more: all but a fraction e^-64 of the base's
 * samples) of both sides in LDS, then streams 16-byte vectors.  Elements
 * beyond are entered by a wave vote: the side's further cells from global
 * memory, and from v_top on the large-v form a + c0 + c1/a + c2/a^2.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include "qm_device.hpp"
#include "qm_hyp_table.h"
#include "qm_internal.h"

namespace qm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int HYP_ROW = HYP_DEGREE + 1;

struct HypSideParams {
    double v0, inv_v0;
    double v_lds, v_top;          /* a < v_lds: LDS cells; a >= v_top: large-v form */
    double c0, c1, c2;
    const double* gcoef;          /* the side's rows in global memory */
    int nlds, ncell;
    int lds_base;                 /* first LDS row of the side */
    int pad;
};

struct HypParams {
    HypSideParams r, l;           /* v >= 0, v < 0 */
    double mu;
    int lds_stride;               /* doubles per LDS row */
    int pad;
};

template <typename T>
struct HypArgs {
    const T* in;
    T* out;
    uint64_t head, nvec, tail_begin, n;
    HypParams P;
};

/* Cell j of t = a / v0 >= 0 (uniform on [0, 1), HYP_SUB per octave beyond)
   and its centre in units of v0.  The centre, 2^k (1 + (i + 1/2)/HYP_SUB),
   is exact, and so is a - centre for a in the cell's octave. */
__device__ __forceinline__ int hyp_cell(double t, double* centre_t)
{
    const bool uni = t < 1.0;
    const int ex = __builtin_amdgcn_frexp_exp(t);           /* t = m 2^ex, m in [0.5, 1) */
    const double m2 = 2.0 * __builtin_amdgcn_frexp_mant(t);  /* [1, 2) */
    const double f = uni ? t : m2 - 1.0;                    /* position in the octave, [0, 1) */
    const int i = (int)(f * HYP_SUB);
    const int k = uni ? 0 : ex - 1;
    const double c = ((uni ? 0.0 : 1.0) + (i + 0.5) * (1.0 / HYP_SUB));
    *centre_t = __builtin_amdgcn_ldexp(c, k);
    return uni ? i : HYP_SUB * (1 + k) + i;
}

__device__ __forceinline__ double hyp_poly(const double* __restrict__ c, double d)
{
    double R = c[0];
#pragma unroll
    for (int k = 1; k <= HYP_DEGREE; ++k) R = __builtin_fma(R, d, c[k]);
    return R;
}

/* a >= v_lds or NaN: global-memory cells up to v_top, then the large-v form. */
static __device__ __noinline__ double hyp_far(double a, const HypSideParams& S)
{
    if (!(a < S.v_top)) {
        if (!(a < __builtin_inf())) return a;                /* inf -> inf, NaN -> NaN */
        return a + (S.c0 + (S.c1 + S.c2 / a) / a);
    }
    double ct;
    int j = hyp_cell(a * S.inv_v0, &ct);
    j = j < S.ncell - 1 ? j : S.ncell - 1;
    j = j > 0 ? j : 0;
    const double d = a - ct * S.v0;
    return a * hyp_poly(S.gcoef + j * HYP_ROW, d);
}

__device__ __forceinline__ double hyp_eval(double v, const double* __restrict__ lds, const HypParams& P)
{
    const bool neg = v < 0.0;
    const double a = __builtin_fabs(v);
    const double v0 = neg ? P.l.v0 : P.r.v0;
    const double inv_v0 = neg ? P.l.inv_v0 : P.r.inv_v0;
    const double v_lds = neg ? P.l.v_lds : P.r.v_lds;
    const int nlds = neg ? P.l.nlds : P.r.nlds;
    const int base = neg ? P.l.lds_base : P.r.lds_base;
    double ct;
    int j = hyp_cell(a * inv_v0, &ct);
    j = j < nlds - 1 ? j : nlds - 1;                         /* far and NaN lanes stay in bounds */
    j = j > 0 ? j : 0;
    const double d = a - ct * v0;
    double Q = a * hyp_poly(lds + (base + j) * P.lds_stride, d);
    const bool far = !(a < v_lds);
    if (wave_any(far)) {
        double qf = hyp_far(far ? a : 0.0, neg ? P.l : P.r);
        Q = far ? qf : Q;
    }
    return P.mu + __builtin_copysign(Q, v);
}

/* Both sides' LDS rows, row stride P.lds_stride. */
__device__ __forceinline__ void stage_hyp(double* lds, const HypParams& P)
{
    const int nr = P.r.nlds * HYP_ROW, nl = P.l.nlds * HYP_ROW;
    for (int i = threadIdx.x; i < nr + nl; i += blockDim.x) {
        const bool left = i >= nr;
        const int e = left ? i - nr : i;
        const int row = e / HYP_ROW, col = e - row * HYP_ROW;
        const double* src = left ? P.l.gcoef : P.r.gcoef;
        lds[((left ? P.l.lds_base : P.r.lds_base) + row) * P.lds_stride + col] = src[e];
    }
}

template <typename T> struct hvec;
template <> struct hvec<double> { typedef d2 type; static constexpr int n = 2; };
template <> struct hvec<float> { typedef f4 type; static constexpr int n = 4; };

/* FP32 in/out: the FP64 evaluation, rounded once. */
template <typename T>
__device__ __forceinline__ T hyp_op(T v, const double* lds, const HypParams& P)
{
    return (T)hyp_eval((double)v, lds, P);
}

template <typename T, bool VECTOR, int UNROLL>
__global__ __launch_bounds__(256) void k_hyperbolic(HypArgs<T> a)
{
    extern __shared__ double lds_hyp[];
    const HypParams P = a.P;
    stage_hyp(lds_hyp, P);
    __syncthreads();

    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VECTOR) {
        typedef typename hvec<T>::type V;
        constexpr int NV = hvec<T>::n;
        const V* vin = reinterpret_cast<const V*>(a.in + a.head);
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        uint64_t i = tid;
        for (; i + (UNROLL - 1) * stride < a.nvec; i += UNROLL * stride) {
            V x[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) x[k] = __builtin_nontemporal_load(vin + i + k * stride);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = hyp_op<T>(x[k][j], lds_hyp, P);
                __builtin_nontemporal_store(y, vout + i + k * stride);
            }
        }
        for (; i < a.nvec; i += stride) {
            V x = __builtin_nontemporal_load(vin + i);
            V y;
#pragma unroll
            for (int j = 0; j < NV; ++j) y[j] = hyp_op<T>(x[j], lds_hyp, P);
            __builtin_nontemporal_store(y, vout + i);
        }
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                a.out[idx] = hyp_op<T>(a.in[idx], lds_hyp, P);
            }
        }
    } else {
        for (uint64_t i = tid; i < a.n; i += stride) a.out[i] = hyp_op<T>(a.in[i], lds_hyp, P);
    }
}

/* LDS row stride: rows of 12 doubles start 24 banks apart; one double of
   padding staggers rows that share a bank.  QM_HYP_LDS_STRIDE (12..20)
   overrides it (tuning). */
static int hyp_lds_stride()
{
    static const int s = [] {
        const char* e = getenv("QM_HYP_LDS_STRIDE");
        int v = e ? atoi(e) : HYP_ROW + 1;
        return (v >= HYP_ROW && v <= 20) ? v : HYP_ROW + 1;
    }();
    return s;
}

constexpr size_t HYP_LDS_MAX = 48 * 1024;   /* bytes of LDS per workgroup for the cells */

static bool side_valid(const HypSide& s, uint64_t ncoef)
{
    return s.noct >= 0 && s.noct <= HYP_MAX_OCT && s.ncell == HYP_SUB * (s.noct + 1) &&
           s.coef_offset + (uint64_t)s.ncell * HYP_ROW <= ncoef && s.v0 > 0 && s.v_top > 0;
}

/* Cells of a side kept in LDS: through the octave that reaches 64 / rate,
   within the LDS budget `cap` rows. */
static int lds_cells(const HypSide& s, double rate, int cap)
{
    int noct = 0;
    while (noct < s.noct && s.v0 * (double)(1ull << noct) < 64.0 / rate) ++noct;
    int n = HYP_SUB * (noct + 1);
    if (n > cap) n = cap - cap % HYP_SUB;
    return n < HYP_SUB ? HYP_SUB : n;
}

static void side_params(const HypSide& s, const double* d_block, int nlds, int base, HypSideParams* p)
{
    p->v0 = s.v0;
    p->inv_v0 = s.inv_v0;
    p->v_top = s.v_top;
    p->v_lds = nlds >= s.ncell ? s.v_top : s.v0 * (double)(1ull << (nlds / HYP_SUB - 1));
    p->c0 = s.far_c0;
    p->c1 = s.far_c1;
    p->c2 = s.far_c2;
    p->gcoef = d_block + s.coef_offset;
    p->nlds = nlds;
    p->ncell = s.ncell;
    p->lds_base = base;
    p->pad = 0;
}

template <typename T>
static hipError_t launch_h(const void* in, void* out, uint64_t n, const HypParams& P, size_t lds, hipStream_t s,
                           const KernelShape& shape)
{
    HypArgs<T> a;
    a.in = static_cast<const T*>(in);
    a.out = static_cast<T*>(out);
    a.n = n;
    a.P = P;
    uintptr_t pin = reinterpret_cast<uintptr_t>(in), pout = reinterpret_cast<uintptr_t>(out);
    constexpr int NV = hvec<T>::n;
    bool coaligned = ((pin - pout) % 16) == 0;
    uint64_t head = coaligned ? ((16 - (pin % 16)) % 16) / sizeof(T) : 0;
    if (coaligned && head <= n && (n - head) >= (uint64_t)NV) {
        a.head = head;
        a.nvec = (n - head) / NV;
        a.tail_begin = head + a.nvec * NV;
        uint64_t per_block = 256ull * shape.unroll;
        uint64_t blocks = (a.nvec + per_block - 1) / per_block;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        if (shape.unroll == 4)
            hipLaunchKernelGGL((k_hyperbolic<T, true, 4>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_hyperbolic<T, true, 1>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else
            hipLaunchKernelGGL((k_hyperbolic<T, true, 2>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    } else {
        a.head = 0;
        a.nvec = n;
        a.tail_begin = n;
        uint64_t blocks = (n + 255) / 256;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((k_hyperbolic<T, false, 1>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_hyperbolic(int dtype, int mode, const void* in, void* out, uint64_t n, const HypTableHeader* d_table,
                             const HypTableHeader& h, uint64_t ncoef, double mu, hipStream_t s,
                             const LaunchShape& shape)
{
    if (!side_valid(h.right, ncoef) || !side_valid(h.left, ncoef)) return hipErrorInvalidValue;
    const double* d_block = reinterpret_cast<const double*>(reinterpret_cast<const char*>(d_table) + sizeof(HypTableHeader));
    const int stride = hyp_lds_stride();
    const int cap = (int)(HYP_LDS_MAX / (sizeof(double) * stride)) / 2;
    HypParams P;
    const int nr = lds_cells(h.right, h.alpha - h.beta, cap);
    const int nl = lds_cells(h.left, h.alpha + h.beta, cap);
    side_params(h.right, d_block, nr, 0, &P.r);
    side_params(h.left, d_block, nl, nr, &P.l);
    P.mu = mu;
    P.lds_stride = stride;
    P.pad = 0;
    const size_t lds = (size_t)(nr + nl) * stride * sizeof(double);
    if (dtype == QM_F64 && mode == QM_PLAIN) return launch_h<double>(in, out, n, P, lds, s, shape.hyperbolic[1]);
    if (dtype == QM_F32 && mode == QM_F32_REFINE) return launch_h<float>(in, out, n, P, lds, s, shape.hyperbolic[0]);
    return hipErrorInvalidValue;
}

}  // namespace qm

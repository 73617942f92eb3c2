/*
 * qm_hyp.hip -- exponential -> hyperbolic recycling kernels (Section 8.1).
 *
 * x = mu + sign(v) Q_side(|v|), Q = a R(a), a = |v|, with R the per-cell
 * polynomial of the side (v >= 0: the right map; v < 0: the mirrored left
 * map) built on the host from the recycling ODE (qm_hyp_table.cpp).  Cells
 * are eight per octave of t = 1 + a/v0 (v0 shared by both sides), so the
 * cell index is the exponent and top three mantissa bits of t, and the
 * cell's centre is t with its lower bits replaced: no table search, no
 * per-side selects but a row offset.  Each workgroup stages the cells that
 * reach a = 64 / rate (all but a fraction e^-64 of the base's samples) of
 * both sides in LDS, then streams 16-byte vectors; a lane evaluates all its
 * elements' polynomials (independent chains) before one wave vote admits
 * the rare far elements: the side's further cells from global memory, and
 * from v_top on the large-v form a + c0 + c1/a + c2/a^2.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>

#include "qm_device.hpp"
#include "qm_hyp_table.h"
#include "qm_internal.h"

namespace qm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

/* Rows of DEG + 1 doubles; in LDS one double of padding staggers the rows
   over the banks (rows of 12 or 8 doubles would otherwise start on the
   same few banks). */
template <int DEG> struct HypRow {
    static constexpr int n = DEG + 1;
    static constexpr int lds = DEG + 2;
};
static_assert(HYP_SUB == 8, "the cell index takes the top 3 mantissa bits of t");

/* The far path's parameters of one side. */
struct HypSideFar {
    double v_top, c0, c1, c2;
    const double* gcoef;          /* the side's rows in global memory */
    int ncell, pad;
};

struct HypParams {
    double v0, inv_v0, mu;        /* v0 is shared by both sides */
    HypSideFar r, l;              /* v >= 0, v < 0 */
    int nlds;                     /* cells per side in LDS, right side's first */
    int pad;
};

template <typename T>
struct HypArgs {
    const T* in;
    T* out;
    uint64_t head, nvec, tail_begin, n;
    HypParams P;
};

/* Cell of t = 1 + a/v0 >= 1: the biased exponent and the top three mantissa
   bits of t give j = 8 k + i for t in [2^k (1 + i/8), 2^k (1 + (i+1)/8));
   the cell's centre in t, 2^k (1 + (i + 1/2)/8), is t with the lower
   mantissa bits replaced by 1000...  NaN and inf give j >= 8192. */
__device__ __forceinline__ int hyp_cell(double t, double* tc)
{
    const uint32_t hi = (uint32_t)__double2hiint(t);
    *tc = __hiloint2double((int)((hi & ~((1u << 17) - 1)) | (1u << 16)), 0);
    return (int)(hi >> 17) - (1023 << 3);
}

template <int DEG>
__device__ __forceinline__ double hyp_poly(const double* __restrict__ c, double d)
{
    double R = c[0];
#pragma unroll
    for (int k = 1; k <= DEG; ++k) R = __builtin_fma(R, d, c[k]);
    return R;
}

/* |Q(v)| from the LDS cells; *far for lanes beyond them (and NaN). */
template <int DEG>
__device__ __forceinline__ double hyp_near(double v, const double* __restrict__ lds, const HypParams& P, bool* far)
{
    const double a = __builtin_fabs(v);
    const double t = __builtin_fma(a, P.inv_v0, 1.0);
    double tc;
    int j = hyp_cell(t, &tc);                    /* >= 0: t >= 1 */
    const bool out = !((unsigned)j < (unsigned)P.nlds);
    *far = out;
    j = out ? P.nlds - 1 : j;                     /* far and NaN lanes stay in bounds */
    const int row = j + (v < 0.0 ? P.nlds : 0);
    const double d = __builtin_fma(-P.v0, tc - 1.0, a);   /* a - centre; tc - 1 is exact */
    return a * hyp_poly<DEG>(lds + row * HypRow<DEG>::lds, d);
}

/* |Q(v)| beyond the LDS cells: the side's global-memory cells up to v_top,
   then the large-v form; inf -> inf, NaN -> NaN.  The side's parameters
   come as plain values selected per lane (a reference to a lane-dependent
   side, or a struct passed by value, would put them in scratch memory). */
template <int DEG>
static __device__ __noinline__ double hyp_far(double a, double v0, double inv_v0, double v_top, double c0, double c1,
                                              double c2, const double* gcoef, int ncell)
{
    if (!(a < v_top)) {
        if (!(a < __builtin_inf())) return a;
        return a + (c0 + (c1 + c2 / a) / a);
    }
    double tc;
    int j = hyp_cell(__builtin_fma(a, inv_v0, 1.0), &tc);
    j = (unsigned)j < (unsigned)ncell ? j : ncell - 1;
    return a * hyp_poly<DEG>(gcoef + j * HypRow<DEG>::n, __builtin_fma(-v0, tc - 1.0, a));
}

template <int DEG>
__device__ __forceinline__ double hyp_far_of(double v, const HypParams& P)
{
    const bool neg = v < 0.0;
    return hyp_far<DEG>(__builtin_fabs(v), P.v0, P.inv_v0, neg ? P.l.v_top : P.r.v_top, neg ? P.l.c0 : P.r.c0,
                   neg ? P.l.c1 : P.r.c1, neg ? P.l.c2 : P.r.c2, neg ? P.l.gcoef : P.r.gcoef,
                   neg ? P.l.ncell : P.r.ncell);
}

/* Both sides' LDS rows: right side rows 0..nlds-1, left side after. */
template <int DEG>
__device__ __forceinline__ void stage_hyp(double* lds, const HypParams& P)
{
    constexpr int W = HypRow<DEG>::n;
    const int n = P.nlds * W;
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) {
        const bool left = i >= n;
        const int e = left ? i - n : i;
        const int row = e / W, col = e - row * W;
        lds[((left ? P.nlds : 0) + row) * HypRow<DEG>::lds + col] = (left ? P.l.gcoef : P.r.gcoef)[e];
    }
}

template <typename T> struct hvec;
template <> struct hvec<double> { typedef d2 type; static constexpr int n = 2; };
template <> struct hvec<float> { typedef f4 type; static constexpr int n = 4; };

/* x = mu + sign(v) |Q|, in FP64; FP32 outputs round it once. */
template <typename T>
__device__ __forceinline__ T hyp_out(double q, T v, const HypParams& P)
{
    return (T)(P.mu + __builtin_copysign(q, (double)v));
}

/* The K elements a lane holds: every element's cell polynomial first (K
   independent chains), then one wave vote for the far fix-up. */
template <typename T, int K, int DEG>
__device__ __forceinline__ void hyp_lane(const T (&v)[K], T (&y)[K], const double* lds, const HypParams& P)
{
    double q[K];
    bool far[K];
    bool anyfar = false;
#pragma unroll
    for (int e = 0; e < K; ++e) {
        q[e] = hyp_near<DEG>((double)v[e], lds, P, &far[e]);
        anyfar |= far[e];
    }
    if (wave_any(anyfar)) {
#pragma unroll
        for (int e = 0; e < K; ++e) {
            if (wave_any(far[e])) {
                double qf = hyp_far_of<DEG>(far[e] ? (double)v[e] : 0.0, P);
                q[e] = far[e] ? qf : q[e];
            }
        }
    }
#pragma unroll
    for (int e = 0; e < K; ++e) y[e] = hyp_out<T>(q[e], v[e], P);
}

template <typename T, bool VECTOR, int UNROLL, int DEG>
__global__ __launch_bounds__(256) void k_hyperbolic(HypArgs<T> a)
{
    extern __shared__ double lds_hyp[];
    const HypParams P = a.P;
    stage_hyp<DEG>(lds_hyp, P);
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
            T v[UNROLL * NV], y[UNROLL * NV];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k)
#pragma unroll
                for (int j = 0; j < NV; ++j) v[k * NV + j] = x[k][j];
            hyp_lane<T, UNROLL * NV, DEG>(v, y, lds_hyp, P);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                V o;
#pragma unroll
                for (int j = 0; j < NV; ++j) o[j] = y[k * NV + j];
                __builtin_nontemporal_store(o, vout + i + k * stride);
            }
        }
        for (; i < a.nvec; i += stride) {
            V x = __builtin_nontemporal_load(vin + i);
            T v[NV], y[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) v[j] = x[j];
            hyp_lane<T, NV, DEG>(v, y, lds_hyp, P);
            V o;
#pragma unroll
            for (int j = 0; j < NV; ++j) o[j] = y[j];
            __builtin_nontemporal_store(o, vout + i);
        }
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                T v[1] = {a.in[idx]}, y[1];
                hyp_lane<T, 1, DEG>(v, y, lds_hyp, P);
                a.out[idx] = y[0];
            }
        }
    } else {
        for (uint64_t i = tid; i < a.n; i += stride) {
            T v[1] = {a.in[i]}, y[1];
            hyp_lane<T, 1, DEG>(v, y, lds_hyp, P);
            a.out[i] = y[0];
        }
    }
}

constexpr size_t HYP_LDS_MAX = 48 * 1024;   /* bytes of LDS per workgroup for the cells */

static bool side_valid(const HypSide& s, int degree, uint64_t ncoef)
{
    return s.degree == degree && s.noct >= 1 && s.noct <= HYP_MAX_OCT && s.ncell == HYP_SUB * s.noct &&
           s.coef_offset + (uint64_t)s.ncell * (degree + 1) <= ncoef && s.v0 > 0 && s.v_top > 0;
}

/* Octaves of t = 1 + v/v0 that reach 64 / rate. */
static int octaves_to(double v0, double rate)
{
    int k = 1;
    while (k < HYP_MAX_OCT && v0 * ((double)(1ull << k) - 1.0) < 64.0 / rate) ++k;
    return k;
}

static void side_far(const HypSide& s, const double* d_block, HypSideFar* f)
{
    f->v_top = s.v_top;
    f->c0 = s.far_c0;
    f->c1 = s.far_c1;
    f->c2 = s.far_c2;
    f->gcoef = d_block + s.coef_offset;
    f->ncell = s.ncell;
    f->pad = 0;
}

template <typename T, int DEG>
static hipError_t launch_h(const void* in, void* out, uint64_t n, const HypTableHeader& h, const HypSide& R,
                           const HypSide& L, uint64_t ncoef, const double* d_block, double mu, hipStream_t s,
                           const KernelShape& shape)
{
    if (!side_valid(R, DEG, ncoef) || !side_valid(L, DEG, ncoef) || R.v0 != L.v0 || R.inv_v0 != L.inv_v0)
        return hipErrorInvalidValue;
    /* LDS cells per side: through the octave reaching 64 / rate on either
       side, within both sides' cells and the LDS budget */
    int noct = std::max(octaves_to(R.v0, h.alpha - h.beta), octaves_to(R.v0, h.alpha + h.beta));
    noct = std::min(noct, std::min(R.noct, L.noct));
    noct = std::min(noct, (int)(HYP_LDS_MAX / (2 * HypRow<DEG>::lds * sizeof(double) * HYP_SUB)));
    HypParams P;
    P.v0 = R.v0;
    P.inv_v0 = R.inv_v0;
    P.mu = mu;
    side_far(R, d_block, &P.r);
    side_far(L, d_block, &P.l);
    P.nlds = HYP_SUB * noct;
    P.pad = 0;
    const size_t lds = (size_t)2 * P.nlds * HypRow<DEG>::lds * sizeof(double);
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
            hipLaunchKernelGGL((k_hyperbolic<T, true, 4, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_hyperbolic<T, true, 1, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else
            hipLaunchKernelGGL((k_hyperbolic<T, true, 2, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    } else {
        a.head = 0;
        a.nvec = n;
        a.tail_begin = n;
        uint64_t blocks = (n + 255) / 256;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((k_hyperbolic<T, false, 1, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_hyperbolic(int dtype, int mode, const void* in, void* out, uint64_t n, const HypTableHeader* d_table,
                             const HypTableHeader& h, uint64_t ncoef, double mu, hipStream_t s,
                             const LaunchShape& shape)
{
    const double* d_block = reinterpret_cast<const double*>(reinterpret_cast<const char*>(d_table) + sizeof(HypTableHeader));
    if (dtype == QM_F64 && mode == QM_PLAIN)
        return launch_h<double, HYP_DEGREE>(in, out, n, h, h.right, h.left, ncoef, d_block, mu, s, shape.hyperbolic[1]);
    if (dtype == QM_F32 && mode == QM_F32_REFINE)
        return launch_h<float, HYP_DEGREE_F32>(in, out, n, h, h.right32, h.left32, ncoef, d_block, mu, s,
                                               shape.hyperbolic[0]);
    return hipErrorInvalidValue;
}

}  // namespace qm

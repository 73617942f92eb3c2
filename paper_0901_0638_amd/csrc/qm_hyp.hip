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
 * from v_top on the large-v form a + c0 + c1/a + c2/a^2 (for variance-gamma
 * targets, whose tail carries a power x^(lambda-1), the form with a log Q
 * term, solved by three fixed-point steps).  The same kernel serves the
 * hyperbolic (Section 8.1) and variance-gamma (Section 8.2) tables.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>

#include "qm_hyp_device.hpp"
#include "qm_internal.h"

namespace qm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct HypArgs {
    const T* in;
    T* out;
    uint64_t head, nvec, tail_begin, n;
    HypParams P;
};

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

/* The first lane's value of x, as a wave-uniform (scalar) value. */
__device__ __forceinline__ uint64_t wave_uniform_u64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

/*
 * VECTOR: each wave streams whole tiles of 64 UNROLL consecutive 16-byte
 * vectors (lane l reads vector l of each 1 KB row), the tiles dealt out to
 * the waves of the grid in turn; only the array's last tile can be partial,
 * and whole waves enter it together (the wave votes need every lane).  The
 * unaligned head and the ragged tail are done by workgroup 0.  Otherwise
 * (input and output not co-aligned) a grid-stride loop over elements.
 */
template <typename T, bool VECTOR, int UNROLL, int DEG>
__global__ __launch_bounds__(256) void k_hyperbolic(HypArgs<T> a)
{
    extern __shared__ __attribute__((aligned(16))) double lds_hyp[];
    const HypParams P = a.P;
    stage_hyp<DEG>(lds_hyp, P);
    __syncthreads();

    if (VECTOR) {
        typedef typename hvec<T>::type V;
        constexpr int NV = hvec<T>::n;
        constexpr int K = UNROLL * NV;
        constexpr uint64_t TILE = 64ull * UNROLL;
        const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        const V* vin = reinterpret_cast<const V*>(a.in + a.head);
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        const uint64_t step = (uint64_t)gridDim.x * 4 * TILE;
        uint64_t t = wave_uniform_u64(((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TILE);
        for (; t + TILE <= a.nvec; t += step) {
            T v[K], y[K];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                V x = __builtin_nontemporal_load(vin + t + 64 * k + lane);
#pragma unroll
                for (int j = 0; j < NV; ++j) v[k * NV + j] = x[j];
            }
            hyp_lane<T, K, DEG>(v, y, lds_hyp, P);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                V o;
#pragma unroll
                for (int j = 0; j < NV; ++j) o[j] = y[k * NV + j];
                __builtin_nontemporal_store(o, vout + t + 64 * k + lane);
            }
        }
        if (t < a.nvec) {
            T v[K], y[K];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                const uint64_t idx = t + 64 * k + lane;
                V x = idx < a.nvec ? __builtin_nontemporal_load(vin + idx) : (V)(T)0;
#pragma unroll
                for (int j = 0; j < NV; ++j) v[k * NV + j] = x[j];
            }
            hyp_lane<T, K, DEG>(v, y, lds_hyp, P);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                const uint64_t idx = t + 64 * k + lane;
                V o;
#pragma unroll
                for (int j = 0; j < NV; ++j) o[j] = y[k * NV + j];
                if (idx < a.nvec) __builtin_nontemporal_store(o, vout + idx);
            }
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
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
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
           s.coef_offset + (uint64_t)s.ncell * (degree + 1) <= ncoef && s.v0 > 0 && s.v_top > 0 &&
           (s.origin == 0 || s.origin == 1);
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
    f->clog = s.far_clog;
    f->gcoef = d_block + s.coef_offset;
    f->ncell = s.ncell;
    f->origin = s.origin;
}

bool make_hyp_params(const HypTableHeader& h, bool f32, const HypTableHeader* d_table, uint64_t ncoef, double mu,
                     HypParams* P, size_t* lds_bytes)
{
    const HypSide& R = f32 ? h.right32 : h.right;
    const HypSide& L = f32 ? h.left32 : h.left;
    const int deg = f32 ? HYP_DEGREE_F32 : HYP_DEGREE;
    if (!side_valid(R, deg, ncoef) || !side_valid(L, deg, ncoef) || R.v0 != L.v0 || R.inv_v0 != L.inv_v0)
        return false;
    const double* d_block = reinterpret_cast<const double*>(reinterpret_cast<const char*>(d_table) + sizeof(HypTableHeader));
    const int stride = f32 ? HypRow<HYP_DEGREE_F32>::lds : HypRow<HYP_DEGREE>::lds;
    /* LDS cells per side: through the octave reaching 64 / rate on either
       side, within both sides' cells and the LDS budget */
    int noct = std::max(octaves_to(R.v0, h.alpha - h.beta), octaves_to(R.v0, h.alpha + h.beta));
    noct = std::min(noct, std::min(R.noct, L.noct));
    noct = std::min(noct, (int)(HYP_LDS_MAX / (2 * stride * sizeof(double) * HYP_SUB)));
    P->v0 = R.v0;
    P->inv_v0 = R.inv_v0;
    P->mu = mu;
    side_far(R, d_block, &P->r);
    side_far(L, d_block, &P->l);
    P->nlds = HYP_SUB * noct;
    P->jlo = (R.origin || L.origin) ? HYP_SUB : 0;
    *lds_bytes = (size_t)2 * P->nlds * stride * sizeof(double);
    return true;
}

template <typename T, int DEG>
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
    const bool f32 = dtype == QM_F32 && mode == QM_F32_REFINE;
    if (!f32 && !(dtype == QM_F64 && mode == QM_PLAIN)) return hipErrorInvalidValue;
    HypParams P;
    size_t lds = 0;
    if (!make_hyp_params(h, f32, d_table, ncoef, mu, &P, &lds)) return hipErrorInvalidValue;
    if (f32) return launch_h<float, HYP_DEGREE_F32>(in, out, n, P, lds, s, shape.hyperbolic[0]);
    return launch_h<double, HYP_DEGREE>(in, out, n, P, lds, s, shape.hyperbolic[1]);
}

}  // namespace qm

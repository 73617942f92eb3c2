/*
 * qm_generate.hip -- fused generation and transform: the open uniforms of a
 * Philox4x32-10 stream (qm_philox.hpp) are drawn in registers and mapped
 * (identity, or the normal quantile in any of its forms) before the only
 * memory access, the 16-byte store of the results -- 8 bytes per FP64
 * sample instead of the 16 of a separate generate-then-transform pass
 * (the reuse of uniform streams the paper's maps are built for).
 *
 * Each lane takes whole Philox blocks: one block is one 16-byte vector of
 * outputs (two FP64 or four FP32 samples).  The hybrid quantiles gather
 * their outer elements across the wave exactly as the streaming kernel does
 * (hybrid_eval), so every output is bitwise the one qm_normal_quantile gives
 * for the same uniform.  Outputs before the first block boundary, after the
 * last whole block, or in an output array that is not 16-byte aligned at a
 * block boundary are done one element at a time by the same per-element
 * functions.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

#include "qm_hybrid.hpp"
#include "qm_hyp_device.hpp"
#include "qm_internal.h"
#include "qm_philox.hpp"
#include "qm_student_device.hpp"

namespace qm {

template <typename T>
struct GenArgs {
    T* out;
    uint32_t k0, k1;
    uint64_t first;       /* stream index of out[0] */
    uint64_t head;        /* out[0, head): before the first block boundary */
    uint64_t nvec;        /* whole blocks from out[head] on */
    uint64_t tail_begin;  /* out[tail_begin, n): after the last whole block */
    uint64_t n;
};

template <typename T> struct OpIdentity { __device__ T operator()(T u) const { return u; } };

/* the NV uniforms of block b */
__device__ __forceinline__ void block_uniforms(uint64_t b, uint32_t k0, uint32_t k1, double (&u)[2])
{
    PhiloxWords w = philox4x32_10(b, k0, k1);
    u[0] = open_u53(w.w[0], w.w[1]);
    u[1] = open_u53(w.w[2], w.w[3]);
}
__device__ __forceinline__ void block_uniforms(uint64_t b, uint32_t k0, uint32_t k1, float (&u)[4])
{
    PhiloxWords w = philox4x32_10(b, k0, k1);
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = open_u23(w.w[j]);
}

/* H: the per-element map (Op), or with GATHER the hybrid (HybridNQ64/32). */
/* The first lane's value of x, as a wave-uniform (scalar) value. */
__device__ __forceinline__ uint64_t gen_wave_uniform(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <typename T, int UNROLL, class H, bool GATHER, bool VECTOR>
__global__ __launch_bounds__(256) void k_generate(GenArgs<T> a)
{
    typedef typename vec16<T>::type V;
    constexpr int NV = vec16<T>::n;
    constexpr int K = NV * UNROLL;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VECTOR) {
        const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        __shared__ T outer_buf[GATHER ? 4 : 1][GATHER ? 64 * K : 1];
        T* buf = outer_buf[GATHER ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        const uint64_t block0 = (a.first + a.head) / NV;
        /* wave-contiguous tiles of 64 UNROLL vectors, dealt out to the waves
           in turn; whole waves iterate together, as the gather needs.  Whole
           tiles store without bound tests; in the one partial last tile the
           blocks past the end are drawn but not stored. */
        constexpr uint64_t TILE = 64ull * UNROLL;
        const uint64_t step = (uint64_t)gridDim.x * 4 * TILE;
        auto tile = [&](uint64_t t, auto whole) {
            const uint64_t i = t + lane;
            T u[K], w[K];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                T b[NV];
                block_uniforms(block0 + i + 64 * k, a.k0, a.k1, b);
#pragma unroll
                for (int j = 0; j < NV; ++j) u[NV * k + j] = b[j];
            }
            if constexpr (GATHER) {
                hybrid_eval<T, K, H>(u, w, buf, lane);
            } else {
                H op;
#pragma unroll
                for (int k = 0; k < K; ++k) w[k] = op(u[k]);
            }
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                uint64_t idx = i + 64 * k;
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = w[NV * k + j];
                if (decltype(whole)::value || idx < a.nvec) __builtin_nontemporal_store(y, vout + idx);
            }
        };
        uint64_t t = gen_wave_uniform(((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TILE);
        for (; t + TILE <= a.nvec; t += step) tile(t, std::true_type());
        if (t < a.nvec) tile(t, std::false_type());
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                T u = stream_uniform<T>(a.first + idx, a.k0, a.k1);
                if constexpr (GATHER) a.out[idx] = H::whole(u);
                else a.out[idx] = H()(u);
            }
        }
    } else {
        for (uint64_t i = tid; i < a.n; i += stride) {
            T u = stream_uniform<T>(a.first + i, a.k0, a.k1);
            if constexpr (GATHER) a.out[i] = H::whole(u);
            else a.out[i] = H()(u);
        }
    }
}

template <typename T, class H, bool GATHER>
static hipError_t launch_gen(GenArgs<T> a, hipStream_t s, const LaunchShape& shape_all)
{
    const KernelShape shape = shape_all.generate[sizeof(T) == 8];
    constexpr int NV = vec16<T>::n;
    a.head = (NV - a.first % NV) % NV;
    bool vector = a.head <= a.n && (a.n - a.head) >= (uint64_t)NV &&
                  (reinterpret_cast<uintptr_t>(a.out + a.head) % 16) == 0;
    if (vector) {
        a.nvec = (a.n - a.head) / NV;
        a.tail_begin = a.head + a.nvec * NV;
        uint64_t per_block = 256ull * shape.unroll;
        uint64_t blocks = (a.nvec + per_block - 1) / per_block;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        if (shape.unroll == 4)
            hipLaunchKernelGGL((k_generate<T, 4, H, GATHER, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_generate<T, 1, H, GATHER, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_generate<T, 2, H, GATHER, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    } else {
        a.head = 0;
        a.nvec = 0;
        a.tail_begin = a.n;
        uint64_t blocks = (a.n + 255) / 256;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((k_generate<T, 1, H, GATHER, false>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_generate(int kind, int dtype, int mode, uint32_t seed, uint32_t stream, uint64_t first,
                           void* out, uint64_t n, hipStream_t s, const LaunchShape& shape)
{
    if (dtype == QM_F64) {
        GenArgs<double> a{};
        a.out = static_cast<double*>(out);
        a.k0 = seed;
        a.k1 = stream;
        a.first = first;
        a.n = n;
        if (kind == QM_UNIFORM && mode == QM_PLAIN) return launch_gen<double, OpIdentity<double>, false>(a, s, shape);
        if (kind == QM_NORMAL_QUANTILE && mode == QM_PLAIN) {
            if (shape.compact) return launch_gen<double, HybridNQ64, true>(a, s, shape);
            return launch_gen<double, OpNQ64Plain, false>(a, s, shape);
        }
        if (kind == QM_NORMAL_QUANTILE && mode == QM_PAPER) return launch_gen<double, OpNQ64Paper, false>(a, s, shape);
    } else if (dtype == QM_F32) {
        GenArgs<float> a{};
        a.out = static_cast<float*>(out);
        a.k0 = seed;
        a.k1 = stream;
        a.first = first;
        a.n = n;
        if (kind == QM_UNIFORM && mode == QM_PLAIN) return launch_gen<float, OpIdentity<float>, false>(a, s, shape);
        if (kind == QM_NORMAL_QUANTILE && mode == QM_F32_REFINE) {
            if (shape.compact) return launch_gen<float, HybridNQ32, true>(a, s, shape);
            return launch_gen<float, OpNQ32Refine, false>(a, s, shape);
        }
        if (kind == QM_NORMAL_QUANTILE && mode == QM_PAPER) return launch_gen<float, OpNQ32Paper, false>(a, s, shape);
        if (kind == QM_NORMAL_QUANTILE && mode == QM_PLAIN) return launch_gen<float, OpNQ32Plain, false>(a, s, shape);
    }
    return hipErrorInvalidValue;
}

StudentParams make_params(const TTableHeader& h, const TCells& c, const double* d_rows);


/* Fused uniform -> normal -> Student t.  The quantile stage is the one of
   k_generate (H, gathered per wave with GATHER); each normal then goes
   through student_eval from the LDS table, as in k_student. */
template <typename T, int UNROLL, class H, bool GATHER, bool VECTOR, int DEG>
__global__ __launch_bounds__(256) void k_generate_t(GenArgs<T> a, const double* __restrict__ coef, StudentParams P)
{
    extern __shared__ __attribute__((aligned(16))) double lds_gt[];
    stage_table(lds_gt, coef, P);
    __syncthreads();
    typedef typename vec16<T>::type V;
    constexpr int NV = vec16<T>::n;
    constexpr int K = NV * UNROLL;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    auto tmap = [&](T z) { return (T)student_eval<DEG>((double)z, lds_gt, P); };
    if (VECTOR) {
        const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        __shared__ T outer_buf[GATHER ? 4 : 1][GATHER ? 64 * K : 1];
        T* buf = outer_buf[GATHER ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0];
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        const uint64_t block0 = (a.first + a.head) / NV;
        /* wave-contiguous tiles of 64 UNROLL vectors, as k_generate: whole
           tiles store without bound tests, the one partial last tile draws
           its blocks past the end but does not store them */
        constexpr uint64_t TILE = 64ull * UNROLL;
        const uint64_t step = (uint64_t)gridDim.x * 4 * TILE;
        auto tile = [&](uint64_t t, auto whole) {
            const uint64_t i = t + lane;
            T u[K], w[K];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                T b[NV];
                block_uniforms(block0 + i + 64 * k, a.k0, a.k1, b);
#pragma unroll
                for (int j = 0; j < NV; ++j) u[NV * k + j] = b[j];
            }
            if constexpr (GATHER) {
                hybrid_eval<T, K, H>(u, w, buf, lane);
            } else {
                H op;
#pragma unroll
                for (int k = 0; k < K; ++k) w[k] = op(u[k]);
            }
#pragma unroll
            for (int k = 0; k < K; ++k) w[k] = tmap(w[k]);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                uint64_t idx = i + 64 * k;
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = w[NV * k + j];
                if (decltype(whole)::value || idx < a.nvec) __builtin_nontemporal_store(y, vout + idx);
            }
        };
        uint64_t t = gen_wave_uniform(((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TILE);
        for (; t + TILE <= a.nvec; t += step) tile(t, std::true_type());
        if (t < a.nvec) tile(t, std::false_type());
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                T u = stream_uniform<T>(a.first + idx, a.k0, a.k1);
                T z;
                if constexpr (GATHER) z = H::whole(u);
                else z = H()(u);
                a.out[idx] = tmap(z);
            }
        }
    } else {
        for (uint64_t i = tid; i < a.n; i += stride) {
            T u = stream_uniform<T>(a.first + i, a.k0, a.k1);
            T z;
            if constexpr (GATHER) z = H::whole(u);
            else z = H()(u);
            a.out[i] = tmap(z);
        }
    }
}

/* The two-sided exponential base sample of an open uniform (Section 8.1),
   in FP64: one logarithm of the side's ratio, by the reduced atanh-series
   log of the quantile path (neg_log_unit; about an ulp, a third of the
   instructions of the library log).  The ratio is a product with the
   side's reciprocal mass, selected before one multiply: two IEEE divisions
   on diverged lanes had cost some 20 instructions per sample. */
struct HypBase {
    double p_minus, inv_p_minus, inv_p_plus, inv_rate_minus, inv_rate_plus;
    __device__ __forceinline__ double operator()(double u) const
    {
        const bool neg = u < p_minus;
        const double ratio = (neg ? u : 1.0 - u) * (neg ? inv_p_minus : inv_p_plus);
        /* u = 1 (an FP64 uniform of the top 53-bit value rounds to 1) is the
           base's right end, v = +inf (mapped to +inf) */
        const double l = ratio > 0.0 ? neg_log_unit(ratio) : __builtin_inf();
        return l * (neg ? -inv_rate_minus : inv_rate_plus);
    }
};

/* The base's constants as the fused hyperbolic kernel takes them: p- and p+
   as exp of the table's log masses, their reciprocals, and the reciprocal
   rates 1/(alpha + beta) and 1/(alpha - beta), each one rounding. */
static void hyp_base_constants(const HypTableHeader& h, HypBase* B)
{
    B->p_minus = std::exp(h.log_p_minus);
    B->inv_p_minus = 1.0 / B->p_minus;
    B->inv_p_plus = 1.0 / std::exp(h.log_p_plus);
    B->inv_rate_minus = 1.0 / (h.alpha + h.beta);
    B->inv_rate_plus = 1.0 / (h.alpha - h.beta);
}

/* Fused uniform -> base sample -> hyperbolic: all K elements of a lane
   through the LDS cells, then one wave vote for the far ones (as
   k_hyperbolic). */
template <typename T, int UNROLL, bool VECTOR, int DEG>
__global__ __launch_bounds__(256) void k_generate_h(GenArgs<T> a, HypParams P, HypBase B)
{
    extern __shared__ __attribute__((aligned(16))) double lds_gh[];
    stage_hyp<DEG>(lds_gh, P);
    __syncthreads();
    typedef typename vec16<T>::type V;
    constexpr int NV = vec16<T>::n;
    constexpr int K = NV * UNROLL;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    auto one = [&](T u) {
        const double v = B((double)u);
        return (T)(P.mu + __builtin_copysign(hyp_abs_q<DEG>(v, lds_gh, P), v));
    };
    if (VECTOR) {
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        const uint64_t block0 = (a.first + a.head) / NV;
        const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        /* wave-contiguous tiles, as k_generate (whole tiles unchecked, the
           partial last one checked) */
        constexpr uint64_t TILE = 64ull * UNROLL;
        const uint64_t step = (uint64_t)gridDim.x * 4 * TILE;
        auto tile = [&](uint64_t t, auto whole) {
            const uint64_t i = t + lane;
            double v[K], q[K];
            bool far[K];
            bool anyfar = false;
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                T b[NV];
                /* blocks past the end are drawn but never stored */
                block_uniforms(block0 + i + 64 * k, a.k0, a.k1, b);
#pragma unroll
                for (int j = 0; j < NV; ++j) v[NV * k + j] = B((double)b[j]);
            }
#pragma unroll
            for (int e = 0; e < K; ++e) {
                q[e] = hyp_near<DEG>(v[e], lds_gh, P, &far[e]);
                anyfar |= far[e];
            }
            if (wave_any(anyfar)) {
#pragma unroll
                for (int e = 0; e < K; ++e) {
                    if (wave_any(far[e])) {
                        double qf = hyp_far_of<DEG>(far[e] ? v[e] : 0.0, P);
                        q[e] = far[e] ? qf : q[e];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                uint64_t idx = i + 64 * k;
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = (T)(P.mu + __builtin_copysign(q[NV * k + j], v[NV * k + j]));
                if (decltype(whole)::value || idx < a.nvec) __builtin_nontemporal_store(y, vout + idx);
            }
        };
        uint64_t t = gen_wave_uniform(((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TILE);
        for (; t + TILE <= a.nvec; t += step) tile(t, std::true_type());
        if (t < a.nvec) tile(t, std::false_type());
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                a.out[idx] = one(stream_uniform<T>(a.first + idx, a.k0, a.k1));
            }
        }
    } else {
        for (uint64_t i = tid; i < a.n; i += stride) a.out[i] = one(stream_uniform<T>(a.first + i, a.k0, a.k1));
    }
}

/* Vector geometry of a generate launch (head, whole blocks, tail) and its
   grid; false if the output takes the element-by-element path. */
template <typename T>
static bool gen_geometry(GenArgs<T>& a, const KernelShape& shape, uint64_t* blocks)
{
    constexpr int NV = vec16<T>::n;
    a.head = (NV - a.first % NV) % NV;
    bool vector = a.head <= a.n && (a.n - a.head) >= (uint64_t)NV &&
                  (reinterpret_cast<uintptr_t>(a.out + a.head) % 16) == 0;
    uint64_t b;
    if (vector) {
        a.nvec = (a.n - a.head) / NV;
        a.tail_begin = a.head + a.nvec * NV;
        uint64_t per_block = 256ull * shape.unroll;
        b = (a.nvec + per_block - 1) / per_block;
    } else {
        a.head = 0;
        a.nvec = 0;
        a.tail_begin = a.n;
        b = (a.n + 255) / 256;
    }
    if (b > shape.max_blocks) b = shape.max_blocks;
    *blocks = b < 1 ? 1 : b;
    return vector;
}

template <typename T, class H, bool GATHER, int DEG>
static hipError_t launch_gen_t(GenArgs<T> a, const double* coef, const StudentParams& P, size_t lds, hipStream_t s,
                               const KernelShape& shape)
{
    uint64_t blocks;
    if (gen_geometry(a, shape, &blocks)) {
        if (shape.unroll == 4)
            hipLaunchKernelGGL((k_generate_t<T, 4, H, GATHER, true, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, coef, P);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_generate_t<T, 1, H, GATHER, true, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, coef, P);
        else
            hipLaunchKernelGGL((k_generate_t<T, 2, H, GATHER, true, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, coef, P);
    } else {
        hipLaunchKernelGGL((k_generate_t<T, 1, H, GATHER, false, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, coef, P);
    }
    return hipGetLastError();
}

/* LDS the gather buffer of a generate kernel takes (4 waves x 64 lanes x K) */
template <typename T>
static size_t gather_bytes(int unroll)
{
    return (size_t)4 * 64 * vec16<T>::n * unroll * sizeof(T);
}

constexpr size_t GEN_LDS_MAX = 65536;   /* static + dynamic LDS of a generate workgroup */

hipError_t launch_generate_student(int dtype, int mode, uint32_t seed, uint32_t stream, uint64_t first, void* out,
                                   uint64_t n, const TTableHeader* d_table, const TTableHeader& h, hipStream_t s,
                                   const LaunchShape& shape)
{
    if (h.identity) return launch_generate(QM_NORMAL_QUANTILE, dtype, mode, seed, stream, first, out, n, s, shape);
    const bool f64 = dtype == QM_F64 && mode == QM_PLAIN;
    if (!f64 && !(dtype == QM_F32 && mode == QM_F32_REFINE)) return hipErrorInvalidValue;
    const TCells& c = f64 ? h.f64 : h.f32;
    const double* coef = table_block(d_table) + c.coef_offset;
    const StudentParams P = make_params(h, c, coef);
    const size_t lds = (size_t)c.nlds * P.lds_stride * sizeof(double);
    const KernelShape ks = shape.generate[f64];
    /* the quantile stage gathers per wave when its buffer fits beside the
       table (bitwise the same results either way) */
    const bool gather = shape.compact &&
                        lds + (f64 ? gather_bytes<double>(ks.unroll) : gather_bytes<float>(ks.unroll)) <= GEN_LDS_MAX;
    if (lds > GEN_LDS_MAX) return hipErrorInvalidValue;
    if (f64) {
        GenArgs<double> a{};
        a.out = static_cast<double*>(out);
        a.k0 = seed;
        a.k1 = stream;
        a.first = first;
        a.n = n;
        if (c.degree == T_DEGREE_LOW) {
            if (gather) return launch_gen_t<double, HybridNQ64, true, T_DEGREE_LOW>(a, coef, P, lds, s, ks);
            return launch_gen_t<double, OpNQ64Plain, false, T_DEGREE_LOW>(a, coef, P, lds, s, ks);
        }
        if (gather) return launch_gen_t<double, HybridNQ64, true, T_DEGREE_HIGH>(a, coef, P, lds, s, ks);
        return launch_gen_t<double, OpNQ64Plain, false, T_DEGREE_HIGH>(a, coef, P, lds, s, ks);
    }
    GenArgs<float> a{};
    a.out = static_cast<float*>(out);
    a.k0 = seed;
    a.k1 = stream;
    a.first = first;
    a.n = n;
    if (gather) return launch_gen_t<float, HybridNQ32, true, T_DEGREE_F32>(a, coef, P, lds, s, ks);
    return launch_gen_t<float, OpNQ32Refine, false, T_DEGREE_F32>(a, coef, P, lds, s, ks);
}

template <typename T, int DEG>
static hipError_t launch_gen_h(GenArgs<T> a, const HypParams& P, const HypBase& B, size_t lds, hipStream_t s,
                               const KernelShape& shape)
{
    uint64_t blocks;
    if (gen_geometry(a, shape, &blocks)) {
        if (shape.unroll == 4)
            hipLaunchKernelGGL((k_generate_h<T, 4, true, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, P, B);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_generate_h<T, 1, true, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, P, B);
        else
            hipLaunchKernelGGL((k_generate_h<T, 2, true, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, P, B);
    } else {
        hipLaunchKernelGGL((k_generate_h<T, 1, false, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a, P, B);
    }
    return hipGetLastError();
}

hipError_t launch_generate_hyperbolic(int dtype, int mode, uint32_t seed, uint32_t stream, uint64_t first, void* out,
                                      uint64_t n, const HypTableHeader* d_table, const HypTableHeader& h,
                                      uint64_t ncoef, double mu, hipStream_t s, const LaunchShape& shape)
{
    const bool f32 = dtype == QM_F32 && mode == QM_F32_REFINE;
    if (!f32 && !(dtype == QM_F64 && mode == QM_PLAIN)) return hipErrorInvalidValue;
    HypParams P;
    size_t lds = 0;
    if (!make_hyp_params(h, f32, d_table, ncoef, mu, &P, &lds)) return hipErrorInvalidValue;
    HypBase B;
    hyp_base_constants(h, &B);
    if (f32) {
        GenArgs<float> a{};
        a.out = static_cast<float*>(out);
        a.k0 = seed;
        a.k1 = stream;
        a.first = first;
        a.n = n;
        return launch_gen_h<float, HYP_DEGREE_F32>(a, P, B, lds, s, shape.hyperbolic[0]);
    }
    GenArgs<double> a{};
    a.out = static_cast<double*>(out);
    a.k0 = seed;
    a.k1 = stream;
    a.first = first;
    a.n = n;
    return launch_gen_h<double, HYP_DEGREE>(a, P, B, lds, s, shape.hyperbolic[1]);
}

}  // namespace qm

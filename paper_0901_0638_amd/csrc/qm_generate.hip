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

#include <type_traits>

#include "qm_hybrid.hpp"
#include "qm_internal.h"
#include "qm_philox.hpp"

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
    for (int j = 0; j < 4; ++j) u[j] = open_u24(w.w[j]);
}

/* H: the per-element map (Op), or with GATHER the hybrid (HybridNQ64/32). */
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
        T* buf = outer_buf[GATHER ? (threadIdx.x >> 6) : 0];
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        const uint64_t block0 = (a.first + a.head) / NV;
        /* whole waves iterate together (the bound is tested on the wave's
           first lane), as the gather needs */
        const uint64_t wave_first = tid - lane;
        for (uint64_t i0 = wave_first; i0 < a.nvec; i0 += UNROLL * stride) {
            const uint64_t i = i0 + lane;
            T u[K], w[K];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                T b[NV];
                block_uniforms(block0 + i + k * stride, a.k0, a.k1, b);
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
                uint64_t idx = i + k * stride;
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = w[NV * k + j];
                if (idx < a.nvec) __builtin_nontemporal_store(y, vout + idx);
            }
        }
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
    const KernelShape shape = shape_all.hybrid[sizeof(T) == 8];
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

}  // namespace qm

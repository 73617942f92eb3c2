/*
 * qm_kernels.hip -- streaming elementwise kernels for gfx950.
 *
 * One template covers every (kind, dtype, mode) of the normal quantile and
 * the exponential -> normal map: a grid-stride loop over 16-byte vectors
 * (two doubles or four floats per lane), UNROLL vectors in flight per lane,
 * non-temporal loads and stores (each byte is touched once), and the
 * unaligned head and tail elements handled by the first workgroup.  The
 * Student t kernels (qm_student.hip) and the batch kernel (qm_batch.hip)
 * reuse the same per-element functions.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "qm_device.hpp"
#include "qm_internal.h"

namespace qm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct vec16;
template <> struct vec16<double> { typedef d2 type; static constexpr int n = 2; };
template <> struct vec16<float> { typedef f4 type; static constexpr int n = 4; };

struct OpNQ64Plain { __device__ double operator()(double u) const { return normal_quantile_f64<false>(u); } };
struct OpNQ64Paper { __device__ double operator()(double u) const { return normal_quantile_f64<true>(u); } };
struct OpE64Plain  { __device__ double operator()(double x) const { return exp_to_normal_f64<false>(x); } };
struct OpE64Paper  { __device__ double operator()(double x) const { return exp_to_normal_f64<true>(x); } };
struct OpNQ32Refine { __device__ float operator()(float u) const { return normal_quantile_f32_refine(u); } };
struct OpNQ32Paper  { __device__ float operator()(float u) const { return normal_quantile_f32_paper(u); } };
struct OpNQ32Plain  { __device__ float operator()(float u) const { return normal_quantile_f32_plain(u); } };
struct OpE32Refine  { __device__ float operator()(float x) const { return exp_to_normal_f32_refine(x); } };

/*
 * in/out: the whole arrays.  [0, head) and [tail_begin, n) are done element
 * by element by workgroup 0; [head, tail_begin) is nvec 16-byte vectors,
 * aligned in both arrays (VECTOR = true) -- or, when the two arrays are not
 * co-aligned, the whole range is done element-wise (VECTOR = false, head =
 * 0, nvec = n).
 */
template <typename T>
struct MapArgs {
    const T* in;
    T* out;
    uint64_t head;
    uint64_t nvec;
    uint64_t tail_begin;
    uint64_t n;
};

template <typename T, bool VECTOR, int UNROLL, class Op>
__global__ __launch_bounds__(256) void k_map(MapArgs<T> a)
{
    Op op;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VECTOR) {
        typedef typename vec16<T>::type V;
        constexpr int NV = vec16<T>::n;
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
                for (int j = 0; j < NV; ++j) y[j] = op(x[k][j]);
                __builtin_nontemporal_store(y, vout + i + k * stride);
            }
        }
        for (; i < a.nvec; i += stride) {
            V x = __builtin_nontemporal_load(vin + i);
            V y;
#pragma unroll
            for (int j = 0; j < NV; ++j) y[j] = op(x[j]);
            __builtin_nontemporal_store(y, vout + i);
        }
        /* unaligned head and ragged tail: fewer than 2 vectors' worth */
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                a.out[idx] = op(a.in[idx]);
            }
        }
    } else {
        for (uint64_t i = tid; i < a.n; i += stride) a.out[i] = op(a.in[i]);
    }
}

/*
 * FP64 quantile, plain mode, with the deep-tail piece compacted across the
 * wave.  On inputs with a tail stratum nearly every wave holds a lane with
 * v > 42, so evaluating the tail piece by wave vote costs every lane the
 * sqrt, the (7,7) rational and a division.  Here each lane keeps K = 2 UNROLL
 * elements; the wave counts its tail elements (ballots), writes their v to a
 * per-wave LDS list at prefix-sum positions, evaluates that list with one
 * element per lane (one pass per 64), and reads each result back.  The
 * arithmetic on every element is the same as normal_quantile_f64<false>,
 * so the results are bitwise identical.
 */
template <int UNROLL>
__global__ __launch_bounds__(256) void k_nq64_compact(MapArgs<double> a)
{
    constexpr int K = 2 * UNROLL;
    __shared__ double tail_buf[4][64 * K];
    double* buf = tail_buf[threadIdx.x >> 6];
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const d2* vin = reinterpret_cast<const d2*>(a.in + a.head);
    d2* vout = reinterpret_cast<d2*>(a.out + a.head);
    /* whole waves iterate together: the trip count is uniform per wave because
       the bound is tested on the wave's first lane */
    const uint64_t wave_first = tid - lane;
    for (uint64_t i0 = wave_first; i0 < a.nvec; i0 += UNROLL * stride) {
        const uint64_t i = i0 + lane;
        double u[K], v[K], mag[K];
        bool tl[K];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            uint64_t idx = i + k * stride;
            d2 x = idx < a.nvec ? __builtin_nontemporal_load(vin + idx) : d2{0.5, 0.5};
            u[2 * k] = x[0];
            u[2 * k + 1] = x[1];
        }
        uint64_t cnt = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] = quantile_v(u[k]);
            mag[k] = expcoord_main(v[k]);
            tl[k] = expcoord_needs_tail(v[k]);
            cnt += __popcll(__ballot(tl[k]));
        }
        if (cnt) {
            uint32_t pos[K];
            uint32_t base = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                uint64_t m = __ballot(tl[k]);
                pos[k] = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (tl[k]) buf[pos[k]] = v[k];
                base += (uint32_t)__popcll(m);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (uint32_t r = 0; r < base; r += 64) {
                if (r + lane < base) buf[r + lane] = expcoord_tail(buf[r + lane]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (tl[k]) mag[k] = buf[pos[k]];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            uint64_t idx = i + k * stride;
            d2 y;
            y[0] = quantile_finish(u[2 * k], mag[2 * k]);
            y[1] = quantile_finish(u[2 * k + 1], mag[2 * k + 1]);
            if (idx < a.nvec) __builtin_nontemporal_store(y, vout + idx);
        }
    }
    if (blockIdx.x == 0) {
        uint64_t extra = a.head + (a.n - a.tail_begin);
        for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
            uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
            a.out[idx] = normal_quantile_f64<false>(a.in[idx]);
        }
    }
}

template <typename T, class Op>
static hipError_t launch_op(const void* in, void* out, uint64_t n, hipStream_t s, const LaunchShape& shape)
{
    MapArgs<T> a;
    a.in = static_cast<const T*>(in);
    a.out = static_cast<T*>(out);
    a.n = n;
    uintptr_t pin = reinterpret_cast<uintptr_t>(in), pout = reinterpret_cast<uintptr_t>(out);
    constexpr int NV = vec16<T>::n;
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
        if (std::is_same<Op, OpNQ64Plain>::value && shape.compact) {
            if (shape.unroll == 4)
                hipLaunchKernelGGL((k_nq64_compact<4>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   *reinterpret_cast<MapArgs<double>*>(&a));
            else if (shape.unroll == 1)
                hipLaunchKernelGGL((k_nq64_compact<1>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   *reinterpret_cast<MapArgs<double>*>(&a));
            else
                hipLaunchKernelGGL((k_nq64_compact<2>), dim3((unsigned)blocks), dim3(256), 0, s,
                                   *reinterpret_cast<MapArgs<double>*>(&a));
        } else if (shape.unroll == 4)
            hipLaunchKernelGGL((k_map<T, true, 4, Op>), dim3((unsigned)blocks), dim3(256), 0, s, a);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_map<T, true, 1, Op>), dim3((unsigned)blocks), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_map<T, true, 2, Op>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    } else {
        a.head = 0;
        a.nvec = n;
        a.tail_begin = n;
        uint64_t blocks = (n + 255) / 256;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((k_map<T, false, 1, Op>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_elementwise(int kind, int dtype, int mode, const void* in, void* out, uint64_t n,
                              hipStream_t s, const LaunchShape& shape)
{
    if (kind == QM_NORMAL_QUANTILE) {
        if (dtype == QM_F64 && mode == QM_PLAIN) return launch_op<double, OpNQ64Plain>(in, out, n, s, shape);
        if (dtype == QM_F64 && mode == QM_PAPER) return launch_op<double, OpNQ64Paper>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_F32_REFINE) return launch_op<float, OpNQ32Refine>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_PAPER) return launch_op<float, OpNQ32Paper>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_PLAIN) return launch_op<float, OpNQ32Plain>(in, out, n, s, shape);
    } else if (kind == QM_EXP_TO_NORMAL) {
        if (dtype == QM_F64 && mode == QM_PLAIN) return launch_op<double, OpE64Plain>(in, out, n, s, shape);
        if (dtype == QM_F64 && mode == QM_PAPER) return launch_op<double, OpE64Paper>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_F32_REFINE) return launch_op<float, OpE32Refine>(in, out, n, s, shape);
    }
    return hipErrorInvalidValue;
}

}  // namespace qm

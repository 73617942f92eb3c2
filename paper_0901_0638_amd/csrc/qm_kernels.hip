/*
 * qm_kernels.hip -- streaming elementwise kernels for gfx950.
 *
 * One template covers every (kind, dtype, mode) of the normal quantile and
 * the exponential -> normal map: wave-contiguous tiles of 16-byte vectors
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
#include "qm_hybrid.hpp"
#include "qm_internal.h"

namespace qm {

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

/* The first lane's value of x, as a wave-uniform (scalar) value. */
__device__ __forceinline__ uint64_t wave_uniform(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

/*
 * VECTOR: each wave streams whole tiles of 64 UNROLL consecutive 16-byte
 * vectors (lane l reads vector l of each 1 KB row), the tiles dealt out to
 * the waves of the grid in turn, as in k_hybrid below; only the array's
 * last tile can be partial, and whole waves enter it together (the maps'
 * wave votes need every lane).  The unaligned head and the ragged tail are
 * done by workgroup 0.  Otherwise (input and output not co-aligned) a
 * grid-stride loop over elements.
 */
template <typename T, bool VECTOR, int UNROLL, class Op>
__global__ __launch_bounds__(256) void k_map(MapArgs<T> a)
{
    Op op;
    if (VECTOR) {
        typedef typename vec16<T>::type V;
        constexpr int NV = vec16<T>::n;
        constexpr uint64_t TILE = 64ull * UNROLL;
        const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        const V* vin = reinterpret_cast<const V*>(a.in + a.head);
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        const uint64_t step = (uint64_t)gridDim.x * 4 * TILE;
        uint64_t t = wave_uniform(((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TILE);
        for (; t + TILE <= a.nvec; t += step) {
            V x[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) x[k] = __builtin_nontemporal_load(vin + t + 64 * k + lane);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = op(x[k][j]);
                __builtin_nontemporal_store(y, vout + t + 64 * k + lane);
            }
        }
        if (t < a.nvec) {
            V x[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                const uint64_t idx = t + 64 * k + lane;
                x[k] = idx < a.nvec ? __builtin_nontemporal_load(vin + idx) : (V)(T)0.5;
            }
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                const uint64_t idx = t + 64 * k + lane;
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = op(x[k][j]);
                if (idx < a.nvec) __builtin_nontemporal_store(y, vout + idx);
            }
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
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride)
            a.out[i] = op(a.in[i]);
    }
}

/*
 * The hybrid quantile over a memory stream (see qm_hybrid.hpp).  Each wave
 * streams whole tiles of 64 UNROLL consecutive 16-byte vectors (UNROLL rows
 * of 1 KB, lane l reading vector l of each row), the tiles dealt out to the
 * waves of the grid in turn.  Measured on MI355X (2^28 FP64 and FP32
 * mixtures), these wave-contiguous tiles stream 2-5% faster than the
 * grid-stride layout (lane vectors a whole grid apart), as they do for a
 * plain copy.  Only the last tile of the array can be partial; the
 * unaligned head and the ragged tail elements are done element by element
 * by workgroup 0.
 */
template <typename T, int UNROLL, class H>
__global__ __launch_bounds__(256) void k_hybrid(MapArgs<T> a)
{
    typedef typename vec16<T>::type V;
    constexpr int NV = vec16<T>::n;
    constexpr int K = NV * UNROLL;
    constexpr uint64_t TILE = 64ull * UNROLL;
    __shared__ T outer_buf[4][64 * K];
    T* buf = outer_buf[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const V* vin = reinterpret_cast<const V*>(a.in + a.head);
    V* vout = reinterpret_cast<V*>(a.out + a.head);
    const uint64_t step = (uint64_t)gridDim.x * 4 * TILE;
    uint64_t t = wave_uniform(((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TILE);
    for (; t + TILE <= a.nvec; t += step) {
        T u[K], w[K];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            V x = __builtin_nontemporal_load(vin + t + 64 * k + lane);
#pragma unroll
            for (int j = 0; j < NV; ++j) u[NV * k + j] = x[j];
        }
        hybrid_eval<T, K, H>(u, w, buf, lane);
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            V y;
#pragma unroll
            for (int j = 0; j < NV; ++j) y[j] = w[NV * k + j];
            __builtin_nontemporal_store(y, vout + t + 64 * k + lane);
        }
    }
    if (t < a.nvec) {      /* the one partial tile (whole waves enter together) */
        T u[K], w[K];
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            const uint64_t idx = t + 64 * k + lane;
            V x = idx < a.nvec ? __builtin_nontemporal_load(vin + idx) : (V)(T)0.5;
#pragma unroll
            for (int j = 0; j < NV; ++j) u[NV * k + j] = x[j];
        }
        hybrid_eval<T, K, H>(u, w, buf, lane);
#pragma unroll
        for (int k = 0; k < UNROLL; ++k) {
            const uint64_t idx = t + 64 * k + lane;
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
            a.out[idx] = H::whole(a.in[idx]);
        }
    }
}

template <typename T, class H>
static void launch_hybrid(const MapArgs<T>& a, uint64_t blocks, hipStream_t s, int unroll)
{
    if (unroll == 4)
        hipLaunchKernelGGL((k_hybrid<T, 4, H>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    else if (unroll == 1)
        hipLaunchKernelGGL((k_hybrid<T, 1, H>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_hybrid<T, 2, H>), dim3((unsigned)blocks), dim3(256), 0, s, a);
}

template <typename T, class H, bool HAS>
struct HybridLaunch {
    static bool run(const MapArgs<T>&, uint64_t, hipStream_t, int) { return false; }
};
template <typename T, class H>
struct HybridLaunch<T, H, true> {
    static bool run(const MapArgs<T>& a, uint64_t blocks, hipStream_t s, int unroll)
    {
        launch_hybrid<T, H>(a, blocks, s, unroll);
        return true;
    }
};

template <typename T, class Op>
static hipError_t launch_op(const void* in, void* out, uint64_t n, hipStream_t s, const LaunchShape& shape)
{
    typedef typename HybridOf<Op>::type H;
    const bool gather = shape.compact && !std::is_void<H>::value;
    const KernelShape ks = gather ? shape.hybrid[sizeof(T) == 8] : (sizeof(T) == 8 ? shape.stream : shape.stream32);
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
        uint64_t per_block = 256ull * ks.unroll;
        uint64_t blocks = (a.nvec + per_block - 1) / per_block;
        if (blocks > ks.max_blocks) blocks = ks.max_blocks;
        if (blocks < 1) blocks = 1;
        if (gather && HybridLaunch<T, H, !std::is_void<H>::value>::run(a, blocks, s, ks.unroll)) {
            /* launched the gathering kernel */
        } else if (ks.unroll == 4)
            hipLaunchKernelGGL((k_map<T, true, 4, Op>), dim3((unsigned)blocks), dim3(256), 0, s, a);
        else if (ks.unroll == 1)
            hipLaunchKernelGGL((k_map<T, true, 1, Op>), dim3((unsigned)blocks), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_map<T, true, 2, Op>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    } else {
        a.head = 0;
        a.nvec = n;
        a.tail_begin = n;
        uint64_t blocks = (n + 255) / 256;
        if (blocks > ks.max_blocks) blocks = ks.max_blocks;
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
        if (dtype == QM_F64 && mode == QM_PAPER_T2) return launch_op<double, OpNQ64PaperT2>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_F32_REFINE) return launch_op<float, OpNQ32Refine>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_PAPER) return launch_op<float, OpNQ32Paper>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_PLAIN) return launch_op<float, OpNQ32Plain>(in, out, n, s, shape);
    } else if (kind == QM_EXP_TO_NORMAL) {
        if (dtype == QM_F64 && mode == QM_PLAIN) return launch_op<double, OpE64Plain>(in, out, n, s, shape);
        if (dtype == QM_F64 && mode == QM_PAPER) return launch_op<double, OpE64Paper>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_F32_REFINE) return launch_op<float, OpE32Refine>(in, out, n, s, shape);
        if (dtype == QM_F32 && mode == QM_PLAIN) return launch_op<float, OpE32Plain>(in, out, n, s, shape);
    }
    return hipErrorInvalidValue;
}

}  // namespace qm

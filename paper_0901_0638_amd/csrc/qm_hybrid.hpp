/*
 * qm_hybrid.hpp -- the per-element maps as kernel functors, and the
 * wave-level gather of the hybrid quantiles (shared by the streaming and the
 * generating kernels).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qm_device.hpp"

namespace qm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct vec16;
template <> struct vec16<double> { typedef d2 type; static constexpr int n = 2; };
template <> struct vec16<float> { typedef f4 type; static constexpr int n = 4; };

struct OpNQ64Plain { __device__ double operator()(double u) const { return normal_quantile_f64<false>(u); } };
struct OpNQ64Paper { __device__ double operator()(double u) const { return normal_quantile_f64<true>(u); } };
struct OpNQ64PaperT2 { __device__ double operator()(double u) const { return normal_quantile_f64_t2(u); } };
struct OpE64Plain  { __device__ double operator()(double x) const { return exp_to_normal_f64<false>(x); } };
struct OpE64Paper  { __device__ double operator()(double x) const { return exp_to_normal_f64<true>(x); } };
struct OpNQ32Refine { __device__ float operator()(float u) const { return normal_quantile_f32_refine(u); } };
struct OpNQ32Paper  { __device__ float operator()(float u) const { return normal_quantile_f32_paper(u); } };
struct OpNQ32Plain  { __device__ float operator()(float u) const { return normal_quantile_f32_plain(u); } };
struct OpE32Refine  { __device__ float operator()(float x) const { return exp_to_normal_f32_refine(x); } };
struct OpE32Plain   { __device__ float operator()(float x) const { return (float)exp_to_normal_f64<false>((double)x); } };

/*
 * The hybrid quantiles (FP64 plain, FP32+refine) split each element into
 * the log-free central piece and the outer, exponential-coordinate path.
 * About 10% of uniform draws (and every element of a tail stratum) lie
 * outside the centre, so nearly every wave holds such a lane, and a wave
 * vote would cost every lane the outer path too.  The kernels instead give
 * every element the central piece, then gather the wave's outer elements
 * (hybrid_eval): each lane keeps K elements; the wave counts its outer elements (ballots),
 * writes their u to a per-wave LDS list at prefix-sum positions, evaluates
 * that list with one element per lane (one pass per 64) and reads each
 * result back.  The arithmetic on every element is that of the per-element
 * function (whole), so the results are bitwise identical to it.
 */
struct HybridNQ64 {
    typedef double T;
    /* central result into w; true if the element needs the outer path */
    static __device__ __forceinline__ bool split(double u, double& w)
    {
        double q = u - 0.5;
        w = central_quantile(q);
        return !is_central(q);
    }
    static __device__ __forceinline__ double outer(double u) { return outer_quantile_f64(u); }
    static __device__ __forceinline__ double whole(double u) { return normal_quantile_f64<false>(u); }
};

struct HybridNQ32 {
    typedef float T;
    static __device__ __forceinline__ bool split(float u, float& w)
    {
        double q = (double)u - 0.5;
        w = central_quantile_f32_refine(u - 0.5f, q);
        return !is_central(q);
    }
    static __device__ __forceinline__ float outer(float u) { return outer_quantile_f32_refine(u); }
    static __device__ __forceinline__ float whole(float u) { return normal_quantile_f32_refine(u); }
};

template <class Op> struct HybridOf { typedef void type; };
template <> struct HybridOf<OpNQ64Plain> { typedef HybridNQ64 type; };
template <> struct HybridOf<OpNQ32Refine> { typedef HybridNQ32 type; };

/* The gather step: u[K] per lane in, w[K] out; buf is the wave's LDS list
   of 64 K elements (its address must be wave-uniform).  Every lane of the
   wave must call it together.  Each slot's ballot is taken once, where its
   comparison is made, and kept as a scalar mask: a lane's list position is
   the running count (scalar) plus the set bits of that mask below the lane
   (two mbcnt), and the list address one shift-add from those. */
template <typename T, int K, class H>
__device__ __forceinline__ void hybrid_eval(const T (&u)[K], T (&w)[K], T* buf, uint32_t lane)
{
    bool outer[K];
    uint64_t m[K];
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        outer[k] = H::split(u[k], w[k]);
        m[k] = __ballot(outer[k]);
        cnt += (uint32_t)__popcll(m[k]);
    }
    if (!cnt) return;
    T* slot[K];
    uint32_t base = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m[k] >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m[k], 0u));
        slot[k] = (buf + base) + below;
        if (outer[k]) *slot[k] = u[k];
        base += (uint32_t)__popcll(m[k]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t r = 0; r < base; r += 64) {
        if (r + lane < base) buf[r + lane] = H::outer(buf[r + lane]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (outer[k]) w[k] = *slot[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace qm

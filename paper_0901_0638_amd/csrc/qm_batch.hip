/*
 * qm_batch.hip -- one persistent launch over many requests of mixed kind,
 * dtype, mode and nu.
 *
 * Every request is cut into chunks of hdr->chunk elements; chunks are numbered
 * globally in request order (chunk_base = prefix sum).  Each workgroup
 * repeatedly claims the next chunk from a device counter, finds its request
 * by binary search over chunk_base, and evaluates it with the same
 * per-element functions as the single-request kernels, so every output is
 * bitwise identical to the single call's.  A chunk belongs to one request,
 * so the kind switch and the wave votes inside the maps are uniform across
 * the workgroup.  A Student t or hyperbolic chunk stages its table in LDS
 * unless the workgroup's previous chunk already did.  The loop ends when the counter
 * passes the last chunk, which every workgroup reaches without waiting on
 * any other.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "qm_batch.h"
#include "qm_device.hpp"
#include "qm_hybrid.hpp"
#include "qm_hyp_device.hpp"
#include "qm_student_device.hpp"

namespace qm {

/* 16-byte vectors per lane, BATCH_UNROLL rows in flight per wave (two
   doubles or four floats each), as the streaming kernels read them. */
constexpr int BATCH_UNROLL = 2;

/* The first lane's value of x, as a wave-uniform (scalar) value. */
__device__ __forceinline__ uint64_t wave_first(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

/*
 * The co-aligned 16-byte body of elements [begin, end) of one request:
 * *head elements precede it and *tail_begin follows its nvec vectors (the
 * return value).  Arrays that are not co-aligned have no body (head = n).
 */
template <typename T>
__device__ __forceinline__ uint64_t chunk_body(const T* in, const T* out, uint64_t n, uint64_t* head,
                                               uint64_t* tail_begin)
{
    constexpr int NV = vec16<T>::n;
    const uintptr_t pi = reinterpret_cast<uintptr_t>(in), po = reinterpret_cast<uintptr_t>(out);
    uint64_t h = ((16 - (pi % 16)) % 16) / sizeof(T);
    if ((pi - po) % 16 != 0 || h > n) h = n;
    const uint64_t nvec = (n - h) / NV;
    *head = h;
    *tail_begin = h + nvec * NV;
    return nvec;
}

/*
 * Elements [begin, end) of one request by the whole workgroup, streamed as
 * the single-request kernels stream an array: each wave takes whole tiles
 * of 64 BATCH_UNROLL consecutive 16-byte vectors (lane l reads vector l of
 * each 1 KB row), the tiles dealt out to the workgroup's waves in turn.
 * Only the chunk's last tile can be partial, and whole waves enter it
 * together (the maps' wave votes need every lane).  The elements before the
 * first co-aligned 16-byte boundary and after the last whole vector, or
 * all of them when the arrays are not co-aligned, go one by one.
 */
template <typename T, class F>
__device__ __forceinline__ void chunk_map(const T* __restrict__ in_, T* __restrict__ out_, uint64_t begin,
                                          uint64_t end, F f)
{
    typedef typename vec16<T>::type V;
    constexpr int NV = vec16<T>::n;
    constexpr uint64_t TILE = 64ull * BATCH_UNROLL;
    const T* in = in_ + begin;
    T* out = out_ + begin;
    const uint64_t n = end - begin;
    uint64_t head, tail_begin;
    const uint64_t nvec = chunk_body(in, out, n, &head, &tail_begin);
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const V* vin = reinterpret_cast<const V*>(in + head);
    V* vout = reinterpret_cast<V*>(out + head);
    const uint64_t step = (uint64_t)(blockDim.x >> 6) * TILE;
    uint64_t t = wave_first((uint64_t)(threadIdx.x >> 6) * TILE);
    for (; t + TILE <= nvec; t += step) {
        V x[BATCH_UNROLL];
#pragma unroll
        for (int k = 0; k < BATCH_UNROLL; ++k) x[k] = __builtin_nontemporal_load(vin + t + 64 * k + lane);
#pragma unroll
        for (int k = 0; k < BATCH_UNROLL; ++k) {
            V y;
#pragma unroll
            for (int j = 0; j < NV; ++j) y[j] = f(x[k][j]);
            __builtin_nontemporal_store(y, vout + t + 64 * k + lane);
        }
    }
    if (t < nvec) {
        V x[BATCH_UNROLL];
#pragma unroll
        for (int k = 0; k < BATCH_UNROLL; ++k) {
            const uint64_t idx = t + 64 * k + lane;
            x[k] = idx < nvec ? __builtin_nontemporal_load(vin + idx) : (V)(T)0.5;
        }
#pragma unroll
        for (int k = 0; k < BATCH_UNROLL; ++k) {
            const uint64_t idx = t + 64 * k + lane;
            V y;
#pragma unroll
            for (int j = 0; j < NV; ++j) y[j] = f(x[k][j]);
            if (idx < nvec) __builtin_nontemporal_store(y, vout + idx);
        }
    }
    const uint64_t extra = head + (n - tail_begin);
    for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
        const uint64_t idx = e < head ? e : tail_begin + (e - head);
        out[idx] = f(in[idx]);
    }
}

extern __shared__ __attribute__((aligned(16))) double lds_tab[];

/* One chunk per op.  Each is a separate, non-inlined function so that its
   constants and registers are its own: inlined together, the union of all
   maps' loop-invariant constants would crowd the persistent loop. */
#define QM_CHUNK_FN(NAME, T, EXPR)                                                                  \
    static __device__ __noinline__ void NAME(const void* in, void* out, uint64_t begin, uint64_t end) \
    {                                                                                               \
        chunk_map<T>((const T*)in, (T*)out, begin, end, [](T x) { return EXPR; });                  \
    }
QM_CHUNK_FN(chunk_nq64_paper, double, normal_quantile_f64<true>(x))
QM_CHUNK_FN(chunk_nq32_paper, float, normal_quantile_f32_paper(x))
QM_CHUNK_FN(chunk_nq32_plain, float, normal_quantile_f32_plain(x))
QM_CHUNK_FN(chunk_e64_plain, double, exp_to_normal_f64<false>(x))
QM_CHUNK_FN(chunk_e64_paper, double, exp_to_normal_f64<true>(x))
QM_CHUNK_FN(chunk_e32_refine, float, exp_to_normal_f32_refine(x))
QM_CHUNK_FN(chunk_e32_plain, float, (float)exp_to_normal_f64<false>((double)x))
QM_CHUNK_FN(chunk_copy64, double, x)
QM_CHUNK_FN(chunk_copy32, float, x)
#undef QM_CHUNK_FN

/* LDS list of the hybrid quantiles' gather: 64 K elements per wave (K = 4
   FP64 or 8 FP32 per lane, two 16-byte vectors), 8 KB per workgroup of four
   waves. */
constexpr int GATHER_DOUBLES_PER_WAVE = 64 * 4;

/*
 * Hybrid quantile chunk (FP64 plain, FP32+refine): the streaming kernel's
 * gather (hybrid_eval) over the same wave tiles as chunk_map, so that the
 * outer path runs once per 64 outer elements rather than on every lane of a
 * wave holding one; bitwise the per-element function.  Whole waves enter
 * every tile together, as the gather needs.  Elements outside the
 * co-aligned 16-byte body take the per-element function.
 */
template <typename T, class H>
static __device__ __noinline__ void chunk_hybrid(const void* vin_, void* vout_, uint64_t begin, uint64_t end,
                                                 double* gather)
{
    typedef typename vec16<T>::type V;
    constexpr int NV = vec16<T>::n;
    constexpr int K = NV * BATCH_UNROLL;
    constexpr uint64_t TILE = 64ull * BATCH_UNROLL;
    const T* in = (const T*)vin_ + begin;
    T* out = (T*)vout_ + begin;
    const uint64_t n = end - begin;
    uint64_t head, tail_begin;
    const uint64_t nvec = chunk_body(in, out, n, &head, &tail_begin);
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    T* buf = reinterpret_cast<T*>(gather + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * GATHER_DOUBLES_PER_WAVE);
    const V* vin = reinterpret_cast<const V*>(in + head);
    V* vout = reinterpret_cast<V*>(out + head);
    const uint64_t step = (uint64_t)(blockDim.x >> 6) * TILE;
    for (uint64_t t = wave_first((uint64_t)(threadIdx.x >> 6) * TILE); t < nvec; t += step) {
        T u[K], w[K];
#pragma unroll
        for (int k = 0; k < BATCH_UNROLL; ++k) {
            const uint64_t idx = t + 64 * k + lane;
            V x = idx < nvec ? __builtin_nontemporal_load(vin + idx) : (V)(T)0.5;
#pragma unroll
            for (int j = 0; j < NV; ++j) u[NV * k + j] = x[j];
        }
        hybrid_eval<T, K, H>(u, w, buf, lane);
#pragma unroll
        for (int k = 0; k < BATCH_UNROLL; ++k) {
            const uint64_t idx = t + 64 * k + lane;
            V y;
#pragma unroll
            for (int j = 0; j < NV; ++j) y[j] = w[NV * k + j];
            if (idx < nvec) __builtin_nontemporal_store(y, vout + idx);
        }
    }
    const uint64_t extra = head + (n - tail_begin);
    for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
        const uint64_t idx = e < head ? e : tail_begin + (e - head);
        out[idx] = H::whole(in[idx]);
    }
}

/* Student t from the table in LDS (referenced by symbol, so the loads stay
   LDS loads). */
template <int DEG>
static __device__ __noinline__ void chunk_t64(const void* in, void* out, uint64_t begin, uint64_t end,
                                              const StudentParams P)
{
    chunk_map<double>((const double*)in, (double*)out, begin, end,
                      [&](double z) { return student_eval<DEG>(z, lds_tab, P); });
}

static __device__ __noinline__ void chunk_t32(const void* in, void* out, uint64_t begin, uint64_t end,
                                              const StudentParams P)
{
    chunk_map<float>((const float*)in, (float*)out, begin, end,
                     [&](float z) { return (float)student_eval<T_DEGREE_F32>((double)z, lds_tab, P); });
}

/* Exponential -> hyperbolic from the cells in LDS: mu + sign(v) |Q(v)|, as
   the map kernel forms it. */
static __device__ __noinline__ void chunk_h64(const void* in, void* out, uint64_t begin, uint64_t end,
                                              const HypParams H)
{
    chunk_map<double>((const double*)in, (double*)out, begin, end, [&](double v) {
        return H.mu + __builtin_copysign(hyp_abs_q<HYP_DEGREE>(v, lds_tab, H), v);
    });
}

static __device__ __noinline__ void chunk_h32(const void* in, void* out, uint64_t begin, uint64_t end,
                                              const HypParams H)
{
    chunk_map<float>((const float*)in, (float*)out, begin, end, [&](float v) {
        const double vd = (double)v;
        return (float)(H.mu + __builtin_copysign(hyp_abs_q<HYP_DEGREE_F32>(vd, lds_tab, H), vd));
    });
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch(BatchHeader* hdr, const BatchReq* __restrict__ reqs)
{
    __shared__ uint64_t s_chunk;
    __shared__ double gather[4 * GATHER_DOUBLES_PER_WAVE];
    const double* loaded = nullptr;        /* table currently in LDS (uniform) */
    const uint64_t total = hdr->total_chunks;
    const uint64_t chunk = hdr->chunk;
    const uint32_t nreq = hdr->nreq;
    uint32_t* const left = hdr->left;
    uint32_t* const done = hdr->done;
    for (;;) {
        if (threadIdx.x == 0) s_chunk = atomicAdd(reinterpret_cast<unsigned long long*>(&hdr->counter), 1ull);
        __syncthreads();
        const uint64_t c = s_chunk;
        __syncthreads();
        if (c >= total) break;
        /* last request with chunk_base <= c (every listed request has chunks) */
        uint32_t lo = 0, hi = nreq - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (reqs[mid].chunk_base <= c) lo = mid; else hi = mid - 1;
        }
        const BatchReq& R = reqs[lo];
        const uint64_t begin = (c - R.chunk_base) * chunk;
        const uint64_t end = begin + chunk < R.n ? begin + chunk : R.n;
        switch (R.op) {
        case BOP_NQ64_PLAIN: chunk_hybrid<double, HybridNQ64>(R.in, R.out, begin, end, gather); break;
        case BOP_NQ64_PAPER: chunk_nq64_paper(R.in, R.out, begin, end); break;
        case BOP_NQ32_REFINE: chunk_hybrid<float, HybridNQ32>(R.in, R.out, begin, end, gather); break;
        case BOP_NQ32_PAPER: chunk_nq32_paper(R.in, R.out, begin, end); break;
        case BOP_NQ32_PLAIN: chunk_nq32_plain(R.in, R.out, begin, end); break;
        case BOP_E64_PLAIN: chunk_e64_plain(R.in, R.out, begin, end); break;
        case BOP_E64_PAPER: chunk_e64_paper(R.in, R.out, begin, end); break;
        case BOP_E32_REFINE: chunk_e32_refine(R.in, R.out, begin, end); break;
        case BOP_E32_PLAIN: chunk_e32_plain(R.in, R.out, begin, end); break;
        case BOP_T64:
        case BOP_T32: {
            if (R.P.identity) {
                if (R.op == BOP_T64) chunk_copy64(R.in, R.out, begin, end);
                else chunk_copy32(R.in, R.out, begin, end);
                break;
            }
            if (loaded != R.coef) {
                __syncthreads();
                stage_table(lds_tab, R.coef, R.P);
                __syncthreads();
                loaded = R.coef;
            }
            if (R.op == BOP_T64) {
                if (R.P.row_shift == 4) chunk_t64<T_DEGREE_HIGH>(R.in, R.out, begin, end, R.P);
                else chunk_t64<T_DEGREE_LOW>(R.in, R.out, begin, end, R.P);
            }
            else chunk_t32(R.in, R.out, begin, end, R.P);
            break;
        }
        case BOP_H64:
        case BOP_H32: {
            if (loaded != R.H.r.gcoef) {
                __syncthreads();
                if (R.op == BOP_H64) stage_hyp<HYP_DEGREE>(lds_tab, R.H);
                else stage_hyp<HYP_DEGREE_F32>(lds_tab, R.H);
                __syncthreads();
                loaded = R.H.r.gcoef;
            }
            if (R.op == BOP_H64) chunk_h64(R.in, R.out, begin, end, R.H);
            else chunk_h32(R.in, R.out, begin, end, R.H);
            break;
        }
        default:
            break;
        }
        if (done && R.flagged) {
            /* per-request completion: each thread's stores of the chunk
               reach device scope before the workgroup counts the chunk;
               the workgroup that counts a request's last chunk raises its
               host-visible flag (release at system scope).  Only requests
               of a few chunks are flagged: the fence writes back the L2,
               too dear for every chunk of a large batch */
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0 &&
                __hip_atomic_fetch_add(left + lo, ~0u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 1u)
                __hip_atomic_store(done + lo, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

/*
 * Descriptor memory of the allocation-free batch entry point: a header and
 * up to QM_BATCH_NOALLOC_MAX_REQUESTS records, one copy per GPU, held until
 * the process ends.  Host code never passes the array's name to a kernel or
 * a copy (on the host it is only a stand-in for the symbol): it uses the
 * device address that batch_scratch_address looks up once per device.
 */
static __device__ __align__(256) unsigned char scratch[BATCH_SCRATCH_BYTES];

hipError_t batch_scratch_address(int device, void** out)
{
    static std::mutex mu;
    static void* addr[BATCH_SCRATCH_MAX_DEVICES] = {};
    *out = nullptr;
    if (device < 0 || device >= BATCH_SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   /* the caller makes `device` current */
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_batch(BatchHeader* d_hdr, const BatchReq* d_reqs, size_t lds_bytes, uint64_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch, dim3((unsigned)blocks), dim3(256), lds_bytes, s, d_hdr, d_reqs);
    return hipGetLastError();
}

}  // namespace qm

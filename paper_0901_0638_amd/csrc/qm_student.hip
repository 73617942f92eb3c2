/*
 * qm_student.hip -- normal -> Student t recycling kernels.
 *
 * t = F_nu^{-1}(Phi(z)) = z R(y), y = z^2, with R the per-cell polynomial
 * built on the host from the recycling ODE (qm_table.cpp).  Each workgroup
 * stages the table in LDS once, then streams 16-byte vectors as the other
 * elementwise kernels do.  Per element: the cell index from y = s^2 by one
 * multiply, the offset d = s^2 - y_c by one fused multiply-add (so the full
 * input precision reaches the polynomial: log R grows like y/(2 nu)), the cell's coefficients from LDS, Horner in d, one multiply by
 * z.  Elements beyond the table (|z| > 10, probability below 1e-23 for a
 * normal sample) take the two-term tail formula of Section 3.5 in log space,
 * entered by a wave vote.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include "qm_device.hpp"
#include "qm_internal.h"
#include "qm_student_device.hpp"

namespace qm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct StudentArgs {
    const T* in;
    T* out;
    uint64_t head, nvec, tail_begin, n;
    const double* coef;       /* device table coefficients (ncell * T_STRIDE) */
    StudentParams P;
};

template <typename T> struct svec;
template <> struct svec<double> { typedef d2 type; static constexpr int n = 2; };
template <> struct svec<float> { typedef f4 type; static constexpr int n = 4; };

template <typename T>
__device__ __forceinline__ T student_op(T z, const double* tab, const StudentParams& P)
{
    if (sizeof(T) == 8) return (T)student_eval((double)z, tab, P);
    /* FP32 in/out: the FP64 evaluation rounded once (the input is exact in
       FP64, so y = z^2 is exact and the table's full accuracy carries over) */
    return (T)student_eval((double)z, tab, P);
}

template <typename T, bool VECTOR, int UNROLL>
__global__ __launch_bounds__(256) void k_student(StudentArgs<T> a)
{
    extern __shared__ double lds_tab[];
    const StudentParams P = a.P;
    stage_table(lds_tab, a.coef, P);
    __syncthreads();

    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VECTOR) {
        typedef typename svec<T>::type V;
        constexpr int NV = svec<T>::n;
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
                for (int j = 0; j < NV; ++j) y[j] = student_op<T>(x[k][j], lds_tab, P);
                __builtin_nontemporal_store(y, vout + i + k * stride);
            }
        }
        for (; i < a.nvec; i += stride) {
            V x = __builtin_nontemporal_load(vin + i);
            V y;
#pragma unroll
            for (int j = 0; j < NV; ++j) y[j] = student_op<T>(x[j], lds_tab, P);
            __builtin_nontemporal_store(y, vout + i);
        }
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                a.out[idx] = student_op<T>(a.in[idx], lds_tab, P);
            }
        }
    } else {
        for (uint64_t i = tid; i < a.n; i += stride) a.out[i] = student_op<T>(a.in[i], lds_tab, P);
    }
}

/* nu = +inf: the identity map (Section 3.1, n -> infinity gives Q = z). */
template <typename T>
__global__ __launch_bounds__(256) void k_identity(const T* in, T* out, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

/* LDS row stride in doubles.  Rows of 16 doubles all start on the same
   bank, so lanes reading different cells conflict; one double of padding
   (17) spreads them (measured: nu = 1 from 200 to 271 Gsamples/s).
   QM_T_LDS_STRIDE (16..24) overrides (tuning). */
int student_lds_stride()
{
    static int stride = [] {
        const char* e = getenv("QM_T_LDS_STRIDE");
        int v = e ? atoi(e) : T_STRIDE + 1;
        return (v >= T_STRIDE && v <= 24) ? v : T_STRIDE + 1;
    }();
    return stride;
}

StudentParams make_params(const TTableHeader& h)
{
    StudentParams P;
    P.h = h.h;
    P.inv_h = h.inv_h;
    P.centre_offset = h.centre_offset;
    P.y_max = h.y_max;
    P.log_K = h.log_K;
    P.tail_a = h.tail_a[0];
    P.sqrt_nu = __builtin_sqrt(h.nu);
    P.inv_nu = 1.0 / h.nu;
    P.nu = h.nu;
    P.ncell = h.ncell;
    P.identity = h.identity;
    P.lds_stride = student_lds_stride();
    return P;
}

template <typename T>
static hipError_t launch_t(const void* in, void* out, uint64_t n, const double* d_coef, const TTableHeader& h,
                           hipStream_t s, const LaunchShape& shape)
{
    if (h.identity) {
        uint64_t blocks = (n + 255) / 256;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        hipLaunchKernelGGL((k_identity<T>), dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const T*>(in), static_cast<T*>(out), n);
        return hipGetLastError();
    }
    StudentArgs<T> a;
    a.in = static_cast<const T*>(in);
    a.out = static_cast<T*>(out);
    a.n = n;
    a.coef = d_coef;
    a.P = make_params(h);
    size_t lds = (size_t)h.ncell * a.P.lds_stride * sizeof(double);
    if (lds > 65536) return hipErrorInvalidValue;   /* beyond the dynamic LDS a launch may ask for */
    uintptr_t pin = reinterpret_cast<uintptr_t>(in), pout = reinterpret_cast<uintptr_t>(out);
    constexpr int NV = svec<T>::n;
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
            hipLaunchKernelGGL((k_student<T, true, 4>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_student<T, true, 1>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else
            hipLaunchKernelGGL((k_student<T, true, 2>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    } else {
        a.head = 0;
        a.nvec = n;
        a.tail_begin = n;
        uint64_t blocks = (n + 255) / 256;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((k_student<T, false, 1>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_student(int dtype, int mode, const void* in, void* out, uint64_t n,
                          const TTableHeader* d_table, const TTableHeader& h_table,
                          hipStream_t s, const LaunchShape& shape)
{
    if (h_table.degree != T_DEGREE && !h_table.identity) return hipErrorInvalidValue;
    if (!h_table.identity && (h_table.ncell < 1 || h_table.stride != T_STRIDE)) return hipErrorInvalidValue;
    const double* d_coef = reinterpret_cast<const double*>(reinterpret_cast<const char*>(d_table) + sizeof(TTableHeader));
    if (dtype == QM_F64 && mode == QM_PLAIN) return launch_t<double>(in, out, n, d_coef, h_table, s, shape);
    if (dtype == QM_F32 && mode == QM_F32_REFINE) return launch_t<float>(in, out, n, d_coef, h_table, s, shape);
    return hipErrorInvalidValue;
}

}  // namespace qm

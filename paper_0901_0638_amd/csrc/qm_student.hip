/*
 * qm_student.hip -- normal -> Student t recycling kernels.
 *
 * t = F_nu^{-1}(Phi(z)) = z R(y), y = z^2, with R the per-cell polynomial
 * built on the host from the recycling ODE (qm_table.cpp).  Each workgroup
 * stages the cells of y <= 100 in LDS once, then streams 16-byte vectors as
 * the other elementwise kernels do.  Per element: the cell index from
 * y = s^2 by one multiply, the offset d = s^2 - y_c by one fused
 * multiply-add (so the full input precision reaches the polynomial: log R
 * grows like y/(2 nu)), the cell's coefficients from LDS, Horner in d, one
 * multiply by z.  FP64 outputs use degree-15 cells, FP32 outputs degree-7
 * cells.  Elements beyond (|z| > 10, probability below 1e-23 for a normal
 * sample) are entered by a wave vote: the table's further cells from global
 * memory, then the two-term tail formula of Section 3.5 in log space.
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
    const double* coef;       /* device cell rows (ncell << P.row_shift doubles) */
    StudentParams P;
};

template <typename T> struct svec;
template <> struct svec<double> { typedef d2 type; static constexpr int n = 2; };
template <> struct svec<float> { typedef f4 type; static constexpr int n = 4; };

/* FP32 in/out: the FP64 evaluation of the table's FP32 cells (R to 1e-10)
   rounded once; the input is exact in FP64, so the cell offset carries the
   input's full precision. */
template <typename T, int DEG>
__device__ __forceinline__ T student_op(T z, const double* tab, const StudentParams& P)
{
    return (T)student_eval<DEG>((double)z, tab, P);
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
 * and whole waves enter it together (the far path's wave vote needs every
 * lane).  The unaligned head and the ragged tail are done by workgroup 0.
 * Otherwise (input and output not co-aligned) a grid-stride loop over
 * elements.
 */
template <typename T, bool VECTOR, int UNROLL, int DEG>
__global__ __launch_bounds__(256) void k_student(StudentArgs<T> a)
{
    extern __shared__ __attribute__((aligned(16))) double lds_tab[];
    const StudentParams P = a.P;
    stage_table(lds_tab, a.coef, P);
    __syncthreads();

    if (VECTOR) {
        typedef typename svec<T>::type V;
        constexpr int NV = svec<T>::n;
        constexpr uint64_t TILE = 64ull * UNROLL;
        const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
        const V* vin = reinterpret_cast<const V*>(a.in + a.head);
        V* vout = reinterpret_cast<V*>(a.out + a.head);
        const uint64_t step = (uint64_t)gridDim.x * 4 * TILE;
        uint64_t t = wave_uniform_u64(((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * TILE);
        for (; t + TILE <= a.nvec; t += step) {
            V x[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) x[k] = __builtin_nontemporal_load(vin + t + 64 * k + lane);
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = student_op<T, DEG>(x[k][j], lds_tab, P);
                __builtin_nontemporal_store(y, vout + t + 64 * k + lane);
            }
        }
        if (t < a.nvec) {
            V x[UNROLL];
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                const uint64_t idx = t + 64 * k + lane;
                x[k] = idx < a.nvec ? __builtin_nontemporal_load(vin + idx) : (V)(T)0;
            }
#pragma unroll
            for (int k = 0; k < UNROLL; ++k) {
                const uint64_t idx = t + 64 * k + lane;
                V y;
#pragma unroll
                for (int j = 0; j < NV; ++j) y[j] = student_op<T, DEG>(x[k][j], lds_tab, P);
                if (idx < a.nvec) __builtin_nontemporal_store(y, vout + idx);
            }
        }
        if (blockIdx.x == 0) {
            uint64_t extra = a.head + (a.n - a.tail_begin);
            for (uint64_t e = threadIdx.x; e < extra; e += blockDim.x) {
                uint64_t idx = e < a.head ? e : a.tail_begin + (e - a.head);
                a.out[idx] = student_op<T, DEG>(a.in[idx], lds_tab, P);
            }
        }
    } else {
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride)
            a.out[i] = student_op<T, DEG>(a.in[i], lds_tab, P);
    }
}

/* nu = +inf: the identity map (Section 3.1, n -> infinity gives Q = z). */
template <typename T>
__global__ __launch_bounds__(256) void k_identity(const T* in, T* out, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

/* LDS row stride in doubles for rows of `row` coefficients: even, so that
   every row starts on a 16-byte boundary and is read in 16-byte pieces.
   Defaults: 10 for rows of 8 (five 16-byte groups, an odd number, so
   consecutive rows start in different groups), 16 for rows of 16 (the
   widest, degree-15 sets take up to 480 rows, which must fit the 64 KB a
   launch may use).  QM_T_LDS_STRIDE (16..24) and QM_T8_LDS_STRIDE (8..24),
   even values only, override them (tuning). */
static int stride_from_env(const char* name, int row, int dflt)
{
    const char* e = getenv(name);
    int v = e ? atoi(e) : dflt;
    return (v >= row && v <= 24 && v % 2 == 0) ? v : dflt;
}

int student_lds_stride(int row)
{
    static const int s16 = stride_from_env("QM_T_LDS_STRIDE", T_DEGREE_HIGH + 1, T_DEGREE_HIGH + 1);
    static const int s8 = stride_from_env("QM_T8_LDS_STRIDE", T_DEGREE_LOW + 1, T_DEGREE_LOW + 3);
    return row == T_DEGREE_HIGH + 1 ? s16 : s8;
}

static bool cells_valid(const TCells& c, int degree)
{
    return c.degree == degree && c.stride == degree + 1 && c.nlds >= 1 && c.ncell >= c.nlds;
}

StudentParams make_params(const TTableHeader& h, const TCells& c, const double* d_rows)
{
    StudentParams P;
    P.h = c.h;
    P.inv_h = c.inv_h;
    P.centre_offset = c.centre_offset;
    P.y_lds = c.y_lds;
    P.y_max = c.y_max;
    P.gcoef = d_rows;
    P.log_K = h.log_K;
    P.tail_a = h.tail_a[0];
    P.sqrt_nu = __builtin_sqrt(h.nu);
    P.inv_nu = 1.0 / h.nu;
    P.nu = h.nu;
    P.ncell = c.ncell;
    P.nlds = c.nlds;
    P.identity = h.identity;
    P.row_shift = c.stride == 16 ? 4 : 3;
    P.lds_stride = student_lds_stride(c.stride);
    return P;
}

template <typename T, int DEG>
static hipError_t launch_t(const void* in, void* out, uint64_t n, const double* d_block, const TTableHeader& h,
                           hipStream_t s, const LaunchShape& shape_all)
{
    const KernelShape shape = shape_all.student[sizeof(T) == 8];
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
    const TCells& c = sizeof(T) == 8 ? h.f64 : h.f32;
    a.coef = d_block + c.coef_offset;
    a.P = make_params(h, c, a.coef);
    size_t lds = (size_t)c.nlds * a.P.lds_stride * sizeof(double);
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
            hipLaunchKernelGGL((k_student<T, true, 4, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else if (shape.unroll == 1)
            hipLaunchKernelGGL((k_student<T, true, 1, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
        else
            hipLaunchKernelGGL((k_student<T, true, 2, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    } else {
        a.head = 0;
        a.nvec = n;
        a.tail_begin = n;
        uint64_t blocks = (n + 255) / 256;
        if (blocks > shape.max_blocks) blocks = shape.max_blocks;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((k_student<T, false, 1, DEG>), dim3((unsigned)blocks), dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_student(int dtype, int mode, const void* in, void* out, uint64_t n,
                          const TTableHeader* d_table, const TTableHeader& h_table,
                          hipStream_t s, const LaunchShape& shape)
{
    if (!h_table.identity && !((cells_valid(h_table.f64, T_DEGREE_LOW) || cells_valid(h_table.f64, T_DEGREE_HIGH)) &&
                               cells_valid(h_table.f32, T_DEGREE_F32)))
        return hipErrorInvalidValue;
    const double* d_block = table_block(d_table);
    if (dtype == QM_F64 && mode == QM_PLAIN) {
        if (h_table.identity || h_table.f64.degree == T_DEGREE_LOW)
            return launch_t<double, T_DEGREE_LOW>(in, out, n, d_block, h_table, s, shape);
        return launch_t<double, T_DEGREE_HIGH>(in, out, n, d_block, h_table, s, shape);
    }
    if (dtype == QM_F32 && mode == QM_F32_REFINE)
        return launch_t<float, T_DEGREE_F32>(in, out, n, d_block, h_table, s, shape);
    return hipErrorInvalidValue;
}

}  // namespace qm

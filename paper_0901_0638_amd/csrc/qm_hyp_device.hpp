/*
 * qm_hyp_device.hpp -- device evaluation of the exponential -> hyperbolic
 * tables (Section 8.1; layout in qm_hyp_table.h), shared by the map kernel
 * (qm_hyp.hip) and the batch kernel (qm_batch.hip).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qm_device.hpp"
#include "qm_hyp_table.h"

namespace qm {

/* Rows of DEG + 1 doubles in global memory.  In LDS every row starts on a
   16-byte boundary and is read in 16-byte pieces (ds_read_b128), so lanes
   on different cells either share a 16-byte bank group or none: never a
   half overlap.  The FP64-output cells (degree 11) keep their twelve
   doubles unpadded, six 16-byte reads.  Measured on MI355X (2^26 base
   samples), this took the FP64 map from 283-329 to 361-363 Gs/s against
   the earlier rows of 13 doubles read as 8-byte pairs, whose stride only
   staggered rows over the banks (rows of 12 or 14 doubles read as 8-byte
   pairs ran at 150-233).  The FP32-output cells (degree 7) are stored
   mixed: the constant term as a double (dwords 0-1), the seven higher
   coefficients as floats, highest power first (dwords 2-8), padded to 12
   dwords: two 16-byte reads and one 4-byte read (36 bytes, against 64 for
   eight doubles).  lds is the row stride in doubles.  The dynamic LDS the
   rows live in is declared 16-byte aligned. */
template <int DEG> struct HypRow {
    static constexpr int n = DEG + 1;
    static constexpr int lds = DEG == HYP_DEGREE_F32 ? 6 : DEG + 1;
    static_assert(lds % 2 == 0, "rows must start on 16-byte boundaries");
};
static_assert(HYP_SUB == 8, "the cell index takes the top 3 mantissa bits of t");

/* The far path's parameters of one side. */
struct HypSideFar {
    double v_top, c0, c1, c2, clog;
    const double* gcoef;          /* the side's rows in global memory */
    int ncell;
    int origin;                   /* 1: v < v0 is the origin series of row 0 */
};

struct HypParams {
    double v0, inv_v0, mu;        /* v0 is shared by both sides */
    HypSideFar r, l;              /* v >= 0, v < 0 */
    int nlds;                     /* cells per side in LDS, right side's first */
    int jlo;                      /* first cell the LDS path takes: 0, or HYP_SUB when the sides
                                     hold the origin series (their first octave goes the far way) */
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

/*
 * R of LDS row `row` at d.  FP64-output cells: Horner in FP64.  FP32-output
 * cells: R = c0 + d S(d), S the seven higher terms by Horner in FP32 from
 * float coefficients, c0 and the last step in FP64.  Across every cell the
 * builder produces, |R - c0| stays a small part of |R| (below 6% for the
 * parameters tested), so the FP32 part adds a relative error of about
 * 0.06 x 2^-22 to R, far below the half-ulp of the FP32 result.
 */
template <int DEG>
__device__ __forceinline__ double hyp_cell(const double* __restrict__ lds, int row, double d)
{
    if constexpr (DEG == HYP_DEGREE_F32) {
        typedef float f4v __attribute__((ext_vector_type(4)));
        typedef double d2v __attribute__((ext_vector_type(2)));
        const double* r = lds + row * HypRow<DEG>::lds;
        const d2v a = *reinterpret_cast<const d2v*>(r);            /* c0, then the top two floats */
        const f4v b = *reinterpret_cast<const f4v*>(r + 2);
        const float last = reinterpret_cast<const float*>(r + 4)[0];
        const double c0 = a.x;
        const float f0 = __int_as_float(__double2loint(a.y)), f1 = __int_as_float(__double2hiint(a.y));
        const float df = (float)d;
        float S = __builtin_fmaf(f0, df, f1);
        S = __builtin_fmaf(S, df, b.x);
        S = __builtin_fmaf(S, df, b.y);
        S = __builtin_fmaf(S, df, b.z);
        S = __builtin_fmaf(S, df, b.w);
        S = __builtin_fmaf(S, df, last);
        return __builtin_fma(d, (double)S, c0);
    } else {
        typedef double d2v __attribute__((ext_vector_type(2)));
        const double* r = lds + row * HypRow<DEG>::lds;
        double c[DEG + 1];
#pragma unroll
        for (int k = 0; k < (DEG + 1) / 2; ++k) {
            const d2v x = *reinterpret_cast<const d2v*>(r + 2 * k);
            c[2 * k] = x.x;
            c[2 * k + 1] = x.y;
        }
        return hyp_poly<DEG>(c, d);
    }
}

/* |Q(v)| from the LDS cells; *far for lanes beyond them (and NaN). */
template <int DEG>
__device__ __forceinline__ double hyp_near(double v, const double* __restrict__ lds, const HypParams& P, bool* far)
{
    const double a = __builtin_fabs(v);
    const double t = __builtin_fma(a, P.inv_v0, 1.0);
    double tc;
    int j = hyp_cell(t, &tc);                    /* >= 0: t >= 1 */
    const bool out = !((unsigned)(j - P.jlo) < (unsigned)(P.nlds - P.jlo));
    *far = out;
    j = out ? P.nlds - 1 : j;                     /* far and NaN lanes stay in bounds */
    const int row = j + (v < 0.0 ? P.nlds : 0);
    const double d = __builtin_fma(-P.v0, tc - 1.0, a);   /* a - centre; tc - 1 is exact */
    return a * hyp_cell<DEG>(lds, row, d);
}

/* R in the first octave of a side with the origin series (row 0 of its
   cells, layout in qm_hyp_table.h): R = P0(a) + w (P1(a) + w (P2(a) +
   w P3(a))), w = a^rho; FP32-output cells have no P3.  The terms in w are
   a small part of R near 0, so the library pow's accuracy is ample. */
template <int DEG>
__device__ __forceinline__ double hyp_origin(const double* __restrict__ row, double a)
{
    /* the families in row order, from the highest power of w down, and
       their degrees in v */
    constexpr int NFAM = DEG == HYP_DEGREE ? 4 : 3;
    constexpr int DG64[4] = {0, 1, 2, 4}, DG32[4] = {0, 1, 3, 0};
    const double w = ::pow(a, row[0]);
    double R = 0;
    int k = 1;
#pragma unroll
    for (int n = 0; n < NFAM; ++n) {
        const int dg = DEG == HYP_DEGREE ? DG64[n] : DG32[n];
        double p = 0;
#pragma unroll
        for (int m = 0; m <= dg; ++m, ++k) p = __builtin_fma(p, a, row[k]);
        R = __builtin_fma(R, w, p);
    }
    return R;
}

/* |Q(v)| beyond the LDS cells: the side's global-memory cells up to v_top,
   then the large-v form; inf -> inf, NaN -> NaN; below v0 on a side with the
   origin series, that series.  The side's parameters come as plain values
   selected per lane (a reference to a lane-dependent side, or a struct
   passed by value, would put them in scratch memory). */
template <int DEG>
static __device__ __noinline__ double hyp_far(double a, double v0, double inv_v0, double v_top, double c0, double c1,
                                              double c2, double clog, const double* gcoef, int ncell, int origin)
{
    if (origin && a < v0) return a * hyp_origin<DEG>(gcoef, a);
    if (!(a < v_top)) {
        if (!(a < __builtin_inf())) return a;
        if (clog == 0.0) return a + (c0 + (c1 + c2 / a) / a);
        /* a tail with a power of x: Q = a + c0 + clog log Q + (c1 + c2/Q)/Q,
           three fixed-point steps (each gains a factor clog/Q) */
        double q = a + c0 - clog * neg_log_unit(a);
        for (int i = 0; i < 3; ++i) q = a + c0 - clog * neg_log_unit(q) + (c1 + c2 / q) / q;
        return q;
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
                   neg ? P.l.c1 : P.r.c1, neg ? P.l.c2 : P.r.c2, neg ? P.l.clog : P.r.clog,
                   neg ? P.l.gcoef : P.r.gcoef, neg ? P.l.ncell : P.r.ncell, neg ? P.l.origin : P.r.origin);
}

/* Both sides' LDS rows: right side rows 0..nlds-1, left side after (for
   the FP32-output cells in the mixed layout of HypRow). */
template <int DEG>
__device__ __forceinline__ void stage_hyp(double* lds, const HypParams& P)
{
    constexpr int W = HypRow<DEG>::n;
    const int n = P.nlds * W;
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) {
        const bool left = i >= n;
        const int e = left ? i - n : i;
        const int row = e / W, col = e - row * W;
        const int r = (left ? P.nlds : 0) + row;
        const double c = (left ? P.l.gcoef : P.r.gcoef)[e];
        if constexpr (DEG == HYP_DEGREE_F32) {
            if (col == DEG) lds[r * HypRow<DEG>::lds] = c;
            else reinterpret_cast<float*>(lds)[2 * r * HypRow<DEG>::lds + 2 + col] = (float)c;
        } else {
            lds[r * HypRow<DEG>::lds + col] = c;
        }
    }
}

/* |Q(v)| of one element, with its own wave vote for the far path. */
template <int DEG>
__device__ __forceinline__ double hyp_abs_q(double v, const double* __restrict__ lds, const HypParams& P)
{
    bool far;
    double q = hyp_near<DEG>(v, lds, P, &far);
    if (wave_any(far)) {
        double qf = hyp_far_of<DEG>(far ? v : 0.0, P);
        q = far ? qf : q;
    }
    return q;
}

/* Kernel parameters of a table's cell set for FP64 (f32 = false) or FP32
   outputs (qm_hyp.hip): false if the header is not a valid table of ncoef
   doubles.  *lds_bytes gets the LDS the staged cells take. */
bool make_hyp_params(const HypTableHeader& h, bool f32, const HypTableHeader* d_table, uint64_t ncoef, double mu,
                     HypParams* P, size_t* lds_bytes);

}  // namespace qm

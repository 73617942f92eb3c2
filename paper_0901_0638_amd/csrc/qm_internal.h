/*
 * qm_internal.h -- declarations shared by the library's translation units
 * (not part of the public ABI).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qm.h"
#include "qm_hyp_table.h"
#include "qm_table.h"

namespace qm {

/* Launch geometry of one kernel family: the grid is capped at max_blocks
   workgroups of 256 (grid-stride beyond), each lane keeps `unroll` 16-byte
   vectors in flight (1, 2 or 4). */
struct KernelShape {
    uint64_t max_blocks;
    int unroll;
};

/* Per family, measured on MI355X (launch-shape sweeps over 1..64
   workgroups per CU x 1..4 vectors): light HBM-bound maps stream best from
   few workgroups with deep unrolling, the VALU-heavy hybrid quantiles from
   many. */
struct LaunchShape {
    KernelShape stream;      /* k_map, FP64: exp -> normal, paper mode */
    KernelShape stream32;    /* k_map, FP32: exp -> normal, paper and plain quantiles */
    KernelShape hybrid[2];   /* [0] FP32+refine, [1] FP64 quantile: k_hybrid */
    KernelShape generate[2]; /* [0] FP32, [1] FP64 outputs: k_generate, k_generate_t */
    KernelShape student[2];  /* [0] FP32, [1] FP64 outputs: k_student */
    KernelShape hyperbolic[2]; /* [0] FP32, [1] FP64: k_hyperbolic */
    int compact;             /* quantiles: gather non-central lanes across the wave */
};

/* Elementwise normal quantile / exp -> normal on one stream. */
hipError_t launch_elementwise(int kind, int dtype, int mode, const void* in, void* out, uint64_t n,
                              hipStream_t s, const LaunchShape& shape);

/* Fused Philox4x32-10 generation and transform (qm_generate.hip). */
hipError_t launch_generate(int kind, int dtype, int mode, uint32_t seed, uint32_t stream, uint64_t first,
                           void* out, uint64_t n, hipStream_t s, const LaunchShape& shape);

/* Fused generation chains (qm_generate.hip): the Student t of the normal
   quantile of each uniform, and the hyperbolic map of each uniform's
   two-sided exponential base sample. */
hipError_t launch_generate_student(int dtype, int mode, uint32_t seed, uint32_t stream, uint64_t first, void* out,
                                   uint64_t n, const TTableHeader* d_table, const TTableHeader& h, hipStream_t s,
                                   const LaunchShape& shape);
hipError_t launch_generate_hyperbolic(int dtype, int mode, uint32_t seed, uint32_t stream, uint64_t first, void* out,
                                      uint64_t n, const HypTableHeader* d_table, const HypTableHeader& h,
                                      uint64_t ncoef, double mu, hipStream_t s, const LaunchShape& shape);

/* The coefficient block that follows a device table's header. */
inline const double* table_block(const TTableHeader* d_table)
{
    return reinterpret_cast<const double*>(reinterpret_cast<const char*>(d_table) + sizeof(TTableHeader));
}

/* Launch the Student t map with a device table (qm_student.hip): FP64
   outputs use the table's f64 cells, FP32 outputs its f32 cells. */
hipError_t launch_student(int dtype, int mode, const void* in, void* out, uint64_t n,
                          const TTableHeader* d_table, const TTableHeader& h_table,
                          hipStream_t s, const LaunchShape& shape);

/* Launch the exponential -> hyperbolic map with a device table
   (qm_hyp.hip); ncoef doubles follow the header. */
hipError_t launch_hyperbolic(int dtype, int mode, const void* in, void* out, uint64_t n, const HypTableHeader* d_table,
                             const HypTableHeader& h, uint64_t ncoef, double mu, hipStream_t s,
                             const LaunchShape& shape);

}  // namespace qm

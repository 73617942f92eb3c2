/*
 * qm_internal.h -- declarations shared by the library's translation units
 * (not part of the public ABI).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qm.h"
#include "qm_table.h"

namespace qm {

/* Launch geometry of the streaming kernels. */
struct LaunchShape {
    uint64_t max_blocks;  /* cap on the grid (grid-stride beyond it) */
    int unroll;           /* 16-byte vectors in flight per lane: 1, 2 or 4 */
    int compact;          /* FP64 quantile: gather non-central lanes across the wave */
};

/* Elementwise normal quantile / exp -> normal on one stream. */
hipError_t launch_elementwise(int kind, int dtype, int mode, const void* in, void* out, uint64_t n,
                              hipStream_t s, const LaunchShape& shape);

/* Fused Philox4x32-10 generation and transform (qm_generate.hip). */
hipError_t launch_generate(int kind, int dtype, int mode, uint32_t seed, uint32_t stream, uint64_t first,
                           void* out, uint64_t n, hipStream_t s, const LaunchShape& shape);

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

}  // namespace qm

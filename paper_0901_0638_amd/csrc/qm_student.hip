/*
 * qm_student.hip -- normal -> Student t recycling kernels.
 */
#include "qm_internal.h"

namespace qm {
hipError_t launch_student(int dtype, int mode, const void* in, void* out, uint64_t n,
                          const TTableHeader* d_table, const TTableHeader& h_table,
                          hipStream_t s, const LaunchShape& shape)
{
    (void)dtype; (void)mode; (void)in; (void)out; (void)n; (void)d_table; (void)h_table; (void)s; (void)shape;
    return hipErrorNotSupported;
}
}

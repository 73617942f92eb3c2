/*
 * qm_batch.h -- descriptors of the persistent batch kernel (internal).
 */
#pragma once
#include <stdint.h>

#include "qm_hyp_device.hpp"
#include "qm_internal.h"
#include "qm_student_device.hpp"

namespace qm {

/* Elements per chunk (a workgroup claims one chunk at a time), carried in
   the batch header: QM_CHUNK_MAX unless tuning lowers the floor, when small
   batches get chunks of about total / (4 x workgroups), between these
   bounds (multiples of QM_CHUNK_MIN keep every chunk start 16-byte aligned
   within an aligned request). */
constexpr uint64_t QM_CHUNK_MIN = 2048;
constexpr uint64_t QM_CHUNK_MAX = 32768;

/* Dynamic LDS (the largest Student t or hyperbolic table of the batch) the batch kernel
   may ask for: 64 KB less its static 8 KB gather list and claim slot. */
constexpr size_t QM_BATCH_DYNAMIC_LDS_MAX = 65536 - 8192 - 256;

enum BatchOp : uint32_t {
    BOP_NQ64_PLAIN = 0, BOP_NQ64_PAPER, BOP_NQ32_REFINE, BOP_NQ32_PAPER, BOP_NQ32_PLAIN,
    BOP_E64_PLAIN, BOP_E64_PAPER, BOP_E32_REFINE, BOP_T64, BOP_T32, BOP_H64, BOP_H32, BOP_E32_PLAIN,
};

/* Device block: header, then nreq BatchReq (then, with per-request
   completion, nreq chunk counters). */
struct BatchHeader {
    uint64_t counter;       /* next chunk to claim; 0 at launch */
    uint64_t total_chunks;
    uint32_t nreq;
    uint32_t reserved;
    uint64_t chunk;         /* elements per chunk */
    /* per-request completion (the serving loop), or both NULL: for a
       request marked `flagged`, left[i] holds its unfinished chunks (its
       chunk count at launch, in device memory) and done[i] is a
       host-visible word, 0 at launch, that the workgroup finishing its last
       chunk sets to 1 once every store of the request has reached memory */
    uint32_t* left;
    uint32_t* done;
};

struct BatchReq {
    uint32_t op;            /* BatchOp */
    uint32_t flagged;       /* per-request completion: count this request's chunks and raise its flag */
    const void* in;
    void* out;
    uint64_t n;
    uint64_t chunk_base;    /* global index of the request's first chunk */
    const double* coef;     /* Student t: device cell rows of the request's dtype */
    union {
        StudentParams P;    /* Student t: table parameters */
        HypParams H;        /* exp -> hyperbolic: table parameters (cells of the request's dtype) */
    };
};

/* The allocation-free entry point's device array: one header and
   QM_BATCH_NOALLOC_MAX_REQUESTS records (768 KiB) per GPU. */
constexpr size_t BATCH_SCRATCH_BYTES = sizeof(BatchHeader) + QM_BATCH_NOALLOC_MAX_REQUESTS * sizeof(BatchReq);
constexpr int BATCH_SCRATCH_MAX_DEVICES = 64;

/* Device address of that array on `device`, which must be the current
   device; looked up on the first call per device and kept (qm_init calls
   it). */
hipError_t batch_scratch_address(int device, void** out);

StudentParams make_params(const TTableHeader& h, const TCells& c, const double* d_rows);
hipError_t launch_batch(BatchHeader* d_hdr, const BatchReq* d_reqs, size_t lds_bytes, uint64_t blocks,
                        hipStream_t s);

}  // namespace qm

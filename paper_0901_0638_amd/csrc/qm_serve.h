/*
 * qm_serve.h -- batch launch and serving loop (internal).
 */
#pragma once
#include <stdint.h>

#include "qm_internal.h"

struct DeviceTable;
struct DeviceHypTable;

namespace qm {

struct Server;

/* Validate one request; sets the last error. */
qm_status check_request(const qm_request& r, int* dtype_size_out, bool single_call);
/* Run one validated request on a stream. */
qm_status run_single(qm_ctx* ctx, const qm_request& r, hipStream_t s);
/* Per-nu table of a context (built on first use). */
qm_status get_table(qm_ctx* ctx, double nu, const DeviceTable** out);
/* Per-(alpha, beta, delta) hyperbolic table of a context (built on first use). */
qm_status get_hyp_table(qm_ctx* ctx, double alpha, double beta, double delta, const DeviceHypTable** out);
/* Per-(lambda, alpha, beta) variance-gamma table (the same format). */
qm_status get_vg_table(qm_ctx* ctx, double lambda, double alpha, double beta, const DeviceHypTable** out);
/* The same lookups without building: QM_E_INVAL if the table is not in the
   context yet. */
qm_status find_table(qm_ctx* ctx, double nu, const DeviceTable** out);
qm_status find_base_table(qm_ctx* ctx, bool vg, double p1, double p2, double p3, const DeviceHypTable** out);
const TTableHeader* device_table_ptr(const DeviceTable* t);
const TTableHeader& device_table_hdr(const DeviceTable* t);
const LaunchShape& ctx_shape(const qm_ctx* ctx);
int ctx_device(const qm_ctx* ctx);
uint64_t ctx_budget(const qm_ctx* ctx);
qm_status set_error(qm_status s, const char* msg);

/* Validate and enqueue requests as one persistent launch (done: optional
   event recorded after it).  flags, if not NULL, is a host-coherent array
   with a zero word for each request with n > 0, in request order: the
   launch sets a request's word to 1 once its output is complete. */
qm_status enqueue_batch(qm_ctx* ctx, const qm_request* reqs, uint64_t count, hipStream_t s, hipEvent_t done,
                        uint32_t* flags = nullptr);
void runner_free(qm_ctx* ctx);
void server_stop(Server* s);

}  // namespace qm

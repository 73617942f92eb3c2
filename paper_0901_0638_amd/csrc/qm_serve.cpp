/*
 * qm_serve.cpp -- batch launch and serving loop.
 */
#include "qm_serve.h"

extern "C" {

qm_status qm_run_batch(qm_ctx* ctx, const qm_request* reqs, uint64_t count, void* hip_stream)
{
    (void)ctx; (void)reqs; (void)count; (void)hip_stream;
    return qm::set_error(QM_E_DTYPE, "qm_run_batch: not available in this build");
}

qm_status qm_submit(qm_ctx* ctx, const qm_request* req, uint64_t* ticket)
{
    (void)ctx; (void)req; (void)ticket;
    return qm::set_error(QM_E_DTYPE, "qm_submit: not available in this build");
}

qm_status qm_poll(qm_ctx* ctx, uint64_t ticket)
{
    (void)ctx; (void)ticket;
    return qm::set_error(QM_E_TICKET, "qm_poll: unknown ticket");
}

uint64_t qm_serving_latencies(qm_ctx* ctx, uint64_t* lat_ns, uint64_t cap)
{
    (void)ctx; (void)lat_ns; (void)cap;
    return 0;
}

}

namespace qm {
void server_stop(Server* s) { (void)s; }
}

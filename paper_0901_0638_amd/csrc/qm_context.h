/*
 * qm_context.h -- the library context (internal).
 */
#pragma once
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "qm_internal.h"

namespace qm {
struct Server;
struct BatchRunner;
}

struct DeviceTable {
    qm::TTableHeader hdr;
    qm::TTableHeader* d_table = nullptr;  /* header followed by coefficients */
};

struct DeviceHypTable {
    qm::HypTableHeader hdr;
    qm::HypTableHeader* d_table = nullptr;  /* header followed by both sides' rows */
    uint64_t ncoef = 0;
};

struct qm_ctx {
    int device = 0;
    uint64_t budget = 0;
    qm::LaunchShape shape{};
    std::mutex table_mu;
    std::map<double, DeviceTable> tables;
    std::map<std::tuple<double, double, double>, DeviceHypTable> hyp_tables;  /* (alpha, beta, delta) */
    std::map<std::tuple<double, double, double>, DeviceHypTable> vg_tables;   /* (lambda, alpha, beta) */
    std::mutex server_mu;
    qm::Server* server = nullptr;
    qm::BatchRunner* runner = nullptr;
    int cus = 256;
    /* qm_run_batch_noalloc: the device array of this GPU (looked up at
       init), a pinned host buffer of the same size and the event that
       marks the last upload from it, all set up by qm_init */
    void* noalloc_dev = nullptr;
    void* noalloc_host = nullptr;
    hipEvent_t noalloc_ev = nullptr;
    std::mutex noalloc_mu;
};


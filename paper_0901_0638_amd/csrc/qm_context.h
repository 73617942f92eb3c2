/*
 * qm_context.h -- the library context (internal).
 */
#pragma once
#include <map>
#include <mutex>
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

struct qm_ctx {
    int device = 0;
    uint64_t budget = 0;
    qm::LaunchShape shape{};
    std::mutex table_mu;
    std::map<double, DeviceTable> tables;
    std::mutex server_mu;
    qm::Server* server = nullptr;
    qm::BatchRunner* runner = nullptr;
    int cus = 256;
};


// Host-side handle types and error helpers shared by the C-ABI sources.
// Internal to libccq.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ccq.h"
#include "ccq_plan.h"

namespace ccq {

// set the thread-local message and return code
ccq_status fail(ccq_status code, const char* fmt, ...);
ccq_status ok();
ccq_status hip_fail(hipError_t e, const char* what);

}  // namespace ccq

struct ccq_context {
    int device;
    int cus;
    size_t lds_per_block;
    void* scratch;          // device address of the fixed scratch on this device (null: host only)
    std::string arch;       // gcnArchName ("host" for a host-only context)
    // tuning cache: batch shape key -> (work-item size, median ms)
    std::mutex tune_mu;
    std::map<uint64_t, std::pair<int32_t, float>> tune;
};

struct ccq_table {
    ccq_context* ctx;
    int64_t n_rows;
    std::vector<ccq_column_desc> cols;
};

struct ccq_plan {
    ccq_context* ctx;
    ccq::DevPlan host;      // host copy (device pointers inside)
    ccq::DevPlan* dev;      // device copy, inside `blob`
    void* blob;             // one device allocation: plan, code tables, sets, slot keys
    int grid_fused;
    int64_t max_groups;
    ccq::WsLayout ws;
};

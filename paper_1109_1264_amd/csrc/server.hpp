// server.hpp -- internal entry points of the serving loop.
#pragma once

#include <string>

#include "salt.h"

namespace salt {

// The loop behind salt_serve_trace; *err receives the message of a failure.
salt_status serve_trace_impl(const salt_server_config *cfg, const salt_request *reqs, int32_t count,
                             salt_request_result *res, std::string *err);

// Launch knobs from the tuning table (kind: 0 eval, 1 dot, 2 nrm2, 3 batch).
salt_status tuned_config(int kind, int route, int dtype, int64_t n, salt_launch_config *out);

}  // namespace salt

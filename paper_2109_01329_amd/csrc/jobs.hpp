// Requests as the serving loop hands them to the batched launch
// (library-internal, plain C++ so that the scheduler builds without HIP).
#pragma once

#include <cstdint>

#include "mirng.h"

namespace mirng {

// A request on a device-resident engine of a server: the request starts
// `skip` engine words (Philox4x32-10) or steps (MRG32k3a) past the state
// held in entry `slot` of the server's device engine table.  The skip is
// fixed when the request is admitted, in arrival order, so the values do
// not depend on how requests are later grouped into batches or streams.
struct EngineRef {
    uint32_t slot;
    uint32_t flags;        // kRefEngine: the request names a resident engine
    uint64_t skip[3];      // 192-bit count, little-endian 64-bit limbs
};
constexpr uint32_t kRefEngine = 1u;
static_assert(sizeof(EngineRef) == 32, "engine reference layout");

// One admitted request: the public request (its engine_type, distribution,
// n and out; seed and offset unused when ref names a resident engine).
struct Job {
    mirng_request req;
    EngineRef ref;
};

}  // namespace mirng

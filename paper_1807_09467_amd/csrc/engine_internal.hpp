// Library-internal hooks of the sequence engine used by the serving loop (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

struct rsolve_seq;

namespace rs {

// Move a sequence to another stream.  Only valid while no work of the sequence is in flight.
void seq_set_stream(rsolve_seq* s, hipStream_t st);

}  // namespace rs

// Library-internal hooks of the sequence engine used by the serving loop (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

struct rsolve_seq;

namespace rs {

// Move a sequence to another stream.  Only valid while no work of the sequence is in flight.
void seq_set_stream(rsolve_seq* s, hipStream_t st);

// Allow (default) or forbid the shared offset lists of the banded product for this sequence.
// Building them reads the banded offsets back once per pattern and groups the rows on the host,
// which pays off over long sequences only.
void seq_set_offset_classes(rsolve_seq* s, bool on);

}  // namespace rs

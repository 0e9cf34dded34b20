// Host-side declarations shared by the runtime (fr_runtime.cpp) and the
// serving loop (fr_server.cpp).  Not part of the public C ABI.
#pragma once
#include <stdint.h>

#include <string>

#include "fr.h"

namespace fr {

// What a client of an index needs to batch requests for it.
struct IndexShape {
  uint32_t dim, vocab, k_max;
  uint32_t max_batch, max_clauses, max_literals;  // per fr_search call
  uint32_t n_workspaces;
  uint32_t batch_terms;    // term lists: most distinct terms per search (0: no limit)
  int device;
};
fr_status index_shape(fr_index* ix, IndexShape* out);

// Record `msg` as this thread's fr_last_error() and return `s`.
fr_status set_error(fr_status s, const std::string& msg);

}  // namespace fr

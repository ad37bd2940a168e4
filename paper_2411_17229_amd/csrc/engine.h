// Internal hooks of the index (defined in dade_api.hip) used by the serving loop (serve.hip).
#pragma once

#include "common.h"
#include "dade.h"

namespace dade {

// Device memory counted against the index's HBM budget (DADE_ENOMEM beyond it).
int index_alloc(dade_index* ix, void** p, size_t bytes);
void index_free(dade_index* ix, void* p, size_t bytes);

// Grows the index's search workspace to hold a search of nq queries whose largest K and nprobe
// are k and nprobe (synchronises s if it grows), so that later searches up to those sizes
// enqueue without synchronising; reports the bytes the whole workspace then holds.
int index_prepare_search(dade_index* ix, int64_t nq, int32_t k, int32_t nprobe, const dade_search_opts& o,
                         hipStream_t s, int64_t* workspace_bytes);

int index_dim(const dade_index* ix);

}  // namespace dade

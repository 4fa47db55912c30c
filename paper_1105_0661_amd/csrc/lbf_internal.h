// lbf_internal.h -- block entry points below the C ABI, shared by abi.cpp and
// the server: validation plus dispatch with the caller's choice of staging.
#pragma once
#include <stddef.h>

#include "../../include/lbf.h"

namespace lbf {

// Bytes of staging (the fast workers' channel-major Stokes before the reorder
// into the final order) one channel of this block needs; 0 for a block that
// needs none.  Host arithmetic on a block that check_block accepts.
size_t block_staging_channel_bytes(const lbf_block* b);

// Validate and run one block: staging from the stream-ordered pool when
// stage is NULL, else through cap bytes at stage (the channels in passes).
int run_block(const lbf_block* b, void* stage, size_t cap, void* stream, const char* where);

// Validate and run a batch; stage NULL: pool staging, else stage[j] / cap[j]
// per block.
int run_batch(const lbf_block* b, int n, void* const* stage, const size_t* cap, void* stream, const char* where);

}  // namespace lbf

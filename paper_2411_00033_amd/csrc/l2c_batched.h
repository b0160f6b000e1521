// l2c_batched.h -- grouped launches of the batched forms for ragged batches (l2c_batched.hip).
#pragma once
#include "l2c_internal.h"

namespace l2c {

// The groups of a ragged batch (one plan per group of equal levels, half-leaf and
// direction) in a batched form run as one launch per kernel template shape: every
// group's kb_up, then the kb_top passes in order, then every group's kb_main, each
// launch covering all the groups of its shape.  The descriptors are built once, at
// batch-plan time, from the group plans (whose workspaces must already hold the group's
// items) and the device item arrays; groups with L = 0 are left out.
struct BatGrouped;
hipError_t batched_grouped_make(const l2c_plan_s *const *plans, const ItemArrays *ia, const int64_t *items,
                                int ngroups, BatGrouped **out);
hipError_t batched_grouped_launch(const BatGrouped *g, hipStream_t stream);
void batched_grouped_free(BatGrouped *g);

}  // namespace l2c

// Shared sparse-pass launches for the serving loop (internal, not part of the
// public ABI).  Problems attached to one batcher hand their sparse passes to
// it; passes that are pending at the same time, of the same precision, mode
// and lane-group geometry, run in one grid on the batcher's stream.
#pragma once
#include "bmg.h"

namespace bmg {
struct PassBatcher;
// on the current device; null on failure
PassBatcher *batcher_create();
void batcher_destroy(PassBatcher *b);
// from now on the problem's sparse passes go through b (until detach)
void batcher_attach(bmg_problem *P, PassBatcher *b);
void batcher_detach(bmg_problem *P);
// launches and passes run so far
void batcher_stats(PassBatcher *b, long *launches, long *passes);
}  // namespace bmg

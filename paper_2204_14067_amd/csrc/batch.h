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

// A bmg_solve that advances one outer iteration of Algorithm 1 per step, so
// that one host thread can interleave several solves.  Errors are returned
// as a bmg_status with the thread's bmg_last_error() message set.
struct SolveTask;
// validates the options as bmg_solve does and runs the initialisation
bmg_status solve_task_create(bmg_problem *P, const bmg_options *opt, SolveTask **out);
// one outer iteration; *done = 1 once converged or at max_iter
bmg_status solve_task_step(SolveTask *t, int *done);
// the final objective, statistics and factors (as bmg_solve returns them)
bmg_status solve_task_finish(SolveTask *t, double *W, double *H, int ld, int *k_out, bmg_result *res);
void solve_task_destroy(SolveTask *t);
}  // namespace bmg

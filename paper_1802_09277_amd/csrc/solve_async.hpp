// Asynchronous form of sth_solve, shared by the blocking solve and the
// serving loop.  Each call only enqueues work on the solve's stream; the
// caller waits for that work (stream sync or event) before the next call.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/sth.h"

namespace sth {

// ||f||^2 and the residual norm^2 of the initial guess u to pinned host
// scalars; starts a solve of L_h u = f to rtol within maxit cycles.
int solve_begin(sth_handle* h, const double* f, double* u, double rtol, int maxit, hipStream_t st);

// Reads the last residual norm; enqueues the next V-cycle and its residual
// norm (*more = true) or the final result mapping into u (*more = false).
int solve_continue(sth_handle* h, bool* more);

// After the last enqueued work completed: cycles, relative residual and
// STH_OK / STH_ENOCONV.
int solve_result(sth_handle* h, int* iters, double* relres);

// Graph capture is skipped (iterations launched one kernel at a time) while
// another thread may allocate or free device memory.
void solve_allow_capture(sth_handle* h, bool allow);

// The event to wait for before the next solve_continue, or nullptr for all
// work enqueued on the solve's stream (a speculative solve keeps the next
// cycle queued behind the one whose norm is read).
hipEvent_t solve_wait_event(sth_handle* h);

}  // namespace sth

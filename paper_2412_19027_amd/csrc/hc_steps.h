// Step-wise driving of one bound solver handle (used by the served form).
// A handle is single-threaded: these calls must not overlap for one handle.
#pragma once
#include "hipcone.h"

namespace hc {
int32_t solver_begin(hc_solver* S);             // initial point; HC_OK or an error code
int32_t solver_step(hc_solver* S, int* done);   // one pass of the loop body; *done = 1 at the end
int32_t solver_finish(hc_solver* S);            // completes the stream, fills the timing fields
}  // namespace hc

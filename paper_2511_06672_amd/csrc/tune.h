// Launch-parameter tuner: picks, per kernel knob and operand shape, the fastest of a few launch
// parameters that change only the speed of a kernel, never its results (for instance how many
// candidates one thread of the rotated-matrix generator serves).  The first call for a shape
// times every choice on the caller's stream with HIP events on the real operands; later calls
// reuse the winner.  The cache is shared by every context of the process.
//
// Environment:
//   GCAMPS_AUTOTUNE=0     turns tuning off (every call returns its fallback); on otherwise.
//   GCAMPS_TUNE_FILE=path JSON cache: read when the path is first seen, rewritten after every new
//                         entry.  Inside "entries", one object per line with the fields in this
//                         order: {"knob": "gen_cpt", "prec": 1, "d": 3, "shape": [256, 256],
//                         "choice": 8, "us": [...]}; "us" holds the measured microseconds of each
//                         choice in the call's order ([] in a hand-written entry).  An entry whose
//                         choice is not among the call's choices is timed again.
//   GCAMPS_TRACE_TUNE     prints one line per decision to stderr (source: timed, file or cache).
#pragma once

#include <hip/hip_runtime.h>

#include <functional>

namespace gc {

// run(choice) launches the kernel with that choice on stream s; it may be called several times
// and must leave the same results whatever the choice.  (s0, s1) is the operand shape the knob
// depends on.  Returns the choice to use.
int tuned_choice(hipStream_t s, const char* knob, int prec, int d, int s0, int s1, const int* choices, int nchoices,
                 int fallback, const std::function<void(int)>& run);

}  // namespace gc

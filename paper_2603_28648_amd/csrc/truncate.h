// Truncation of the optimised window and move to the next window.
#pragma once
#include "engine.h"

namespace dmrg {

struct TruncResult {
  double trunc_err = 0;  // discarded weight / total weight
  int kept = 0;          // new bond dimension
  int64_t next_size = 0; // psi size of the next window
};

// Updates m in place: dir = +1 stores the new left-canonical A_window and
// moves the window to window+1; dir = -1 stores the new right-canonical
// B_{window+1} and moves to window-1.  next_psi receives the guess for the
// next window (psi layout of include/dmrg.h).
TruncResult truncate_and_move(Mps& m, int window, const double* psi, int dir, int max_d,
                              double cutoff, DevBuf& next_psi, DevBuf& scratch, hipStream_t s);

}  // namespace dmrg

// Online autotuner of launch configurations (tune.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace slrx {

// Kernel classes with tuned launch configurations.
enum TuneKind {
  TUNE_TRI = 1,       // Householder tridiagonalisation: workgroups per column launch (a = n, b = problems)
  TUNE_CG_GROUP = 2,  // engine step: the CG of each problem on its own stream (0) or grouped launches (1)
                      // (a = problems, b = their summed volume / 4096, c = largest M << 16 | largest n_cg)
  TUNE_TRI_ACCESS = 3,  // tridiagonalisation rows cached (0) or nontemporal (1), once TUNE_TRI has chosen
                        // (a = n, b = problems, c = the chosen TUNE_TRI candidate)
};

// Timing of one call made with a candidate configuration.
struct TuneTicket {
  int key_kind = 0, a = 0, b = 0, c = 0, dev = 0, slot = -1;
  hipEvent_t e1 = nullptr;
};

// The candidate (0 .. ncand-1) to use for this call of the kernel class on a
// shape; while the choice is open, the call is timed between tune_begin and
// tune_end on stream s.  Thread-safe.
int tune_begin(int kind, int a, int b, int c, int ncand, hipStream_t s, TuneTicket& t);
void tune_end(const TuneTicket& t, hipStream_t s);
// The chosen candidate for a shape, or -1 while it is still being tuned.
int tune_choice(int kind, int a, int b, int c);

}  // namespace slrx

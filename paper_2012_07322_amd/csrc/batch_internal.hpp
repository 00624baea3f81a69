// Library-internal view of a batch for the request server: the work items a
// block would add to the batch's lists (so admission can keep every list
// within the batch's capacity), the batch's stream and steps replayed
// several at a time.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/gmunu.h"

namespace gm {

constexpr int kMaxVariants = 32;  // bound on the number of stage work lists

struct BatchItems {
  int variant;  // stage list the block would join (tile variant and Riemann solver)
  long stage;   // items in that stage list
  long cells;   // items in the recovery and CFL lists (256 interior cells each)
  long ghosts;  // items in the ghost list
};

// b may be null: the default tile variant, as for a batch never tuned.
BatchItems batch_items_for(const gmunu_batch *b, const gmunu_grid_desc &d);
long batch_max_items(const gmunu_batch *b);

// The batch's private stream, on which its captured steps replay.  A caller
// that issues all of its work for the batch on this stream saves the events
// that otherwise order the replay against the caller's stream.
hipStream_t batch_stream(const gmunu_batch *b);

// gmunu_batch_step with use_graph set, `steps` whole steps per replay of the
// captured graph (re-captured when steps changes).
int batch_step_graph(gmunu_batch *b, double cfl, unsigned int *nfatal_dev, int steps, hipStream_t st);

}  // namespace gm

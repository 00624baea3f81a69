// Library-internal view of a batch for the request server: the work items a
// block would add to the batch's lists (so admission can keep every list
// within the batch's capacity).
#pragma once

#include "../../include/gmunu.h"

namespace gm {

constexpr int kMaxVariants = 32;  // bound on the number of stage work lists

struct BatchItems {
  int variant;  // stage list the block would join (tile variant and Riemann solver)
  long stage;   // items in that stage list
  long cells;   // items in the recovery and CFL lists (256 interior cells each)
  long ghosts;  // items in the ghost list
};

BatchItems batch_items_for(const gmunu_batch *b, const gmunu_grid_desc &d);
long batch_max_items(const gmunu_batch *b);

}  // namespace gm

// Library-internal view of a batch for the request server: the work items a
// block would add to the batch's lists (so admission can keep every list
// within the batch's capacity).
#pragma once

#include "../../include/gmunu.h"

namespace gm {

struct BatchItems {
  int variant;  // tile variant the block would get (tuned or default)
  long stage;   // items in that variant's stage list
  long cells;   // items in the recovery and CFL lists (256 interior cells each)
  long ghosts;  // items in the ghost list
};

BatchItems batch_items_for(const gmunu_batch *b, const gmunu_grid_desc &d);
long batch_max_items(const gmunu_batch *b);

}  // namespace gm

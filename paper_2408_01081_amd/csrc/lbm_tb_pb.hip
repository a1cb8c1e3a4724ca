// Instantiations of the load-free blocked kernels, periodic lattices, second part of the variant table.
#include <hip/hip_runtime.h>

#include "lbm_tb_tables.hpp"

namespace lbmk {

void tb_fill_periodic_b(TBFn* out) {
  tb_fill_range<LBM_PERIODIC, kTBSplit>(
      out, std::make_integer_sequence<int, kNumTBVariants - kTBSplit>{});
}

}  // namespace lbmk

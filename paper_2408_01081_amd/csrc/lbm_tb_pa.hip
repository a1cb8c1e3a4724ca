// Instantiations of the load-free blocked kernels, periodic lattices, first part of the variant table.
#include <hip/hip_runtime.h>

#include "lbm_tb_tables.hpp"

namespace lbmk {

void tb_fill_periodic_a(TBFn* out) {
  tb_fill_range<LBM_PERIODIC, 0>(out, std::make_integer_sequence<int, kTBSplit>{});
}

}  // namespace lbmk

// Instantiations of the load-free blocked kernels, Dirichlet lattices, second part of the variant table.
#include <hip/hip_runtime.h>

#include "lbm_tb_tables.hpp"

namespace lbmk {

void tb_fill_dirichlet_b(TBFn* out) {
  tb_fill_range<LBM_DIRICHLET, kTBSplit>(
      out, std::make_integer_sequence<int, kNumTBVariants - kTBSplit>{});
}

}  // namespace lbmk

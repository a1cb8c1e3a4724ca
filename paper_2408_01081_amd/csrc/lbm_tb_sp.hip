// Instantiations of the split Dirichlet kernels (wall band and interior in one launch).
#include <hip/hip_runtime.h>

#include "lbm_tb_tables.hpp"

namespace lbmk {

void tb_fill_split(TBSplitFn* out) {
  tbs_fill(out, std::make_integer_sequence<int, kNumTBSplitVariants>{});
}

}  // namespace lbmk

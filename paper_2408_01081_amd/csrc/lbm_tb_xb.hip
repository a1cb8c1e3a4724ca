// Instantiations of the blocked kernels with a body load and/or the displacement state (variants for the steps left over after the last full launch).
#include <hip/hip_runtime.h>

#include "lbm_tb_tables.hpp"

namespace lbmk {

void tb_fill_extra_b(TBExtFns* out) {
  tbx_fill_range<kTBExtSplit>(out,
                              std::make_integer_sequence<int, kNumTBExtVariants - kTBExtSplit>{});
}

}  // namespace lbmk

// Instantiations of the blocked kernels with a body load and/or the displacement state (whole-run variants).
#include <hip/hip_runtime.h>

#include "lbm_tb_tables.hpp"

namespace lbmk {

void tb_fill_extra_a(TBExtFns* out) {
  tbx_fill_range<0>(out, std::make_integer_sequence<int, kTBExtSplit>{});
}

}  // namespace lbmk

// Reduced-precision leaf kernels instantiated for one element format.
#include "leaf_mfma_impl.hpp"

namespace knng {
namespace leafk {
int run_bf16(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err, size_t errlen) {
    return launch_fmt_any<kBF16>(a, rr, launches, err, errlen);
}
}  // namespace leafk
}  // namespace knng

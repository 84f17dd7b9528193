// Instantiations of the workgroup-resident light-cone kernel (see fused_impl.hpp).
#include "fused_impl.hpp"

namespace qaoa {

hipError_t launch_fused_k14(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                          const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    return launch_k<14>(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
}

}  // namespace qaoa

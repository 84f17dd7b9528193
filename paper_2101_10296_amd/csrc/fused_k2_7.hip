// Instantiations of the workgroup-resident light-cone kernel (see fused_impl.hpp).
#include "fused_impl.hpp"

namespace qaoa {

hipError_t launch_fused_k2(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                          const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    return launch_k<2>(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
}

hipError_t launch_fused_k3(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                          const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    return launch_k<3>(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
}

hipError_t launch_fused_k4(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                          const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    return launch_k<4>(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
}

hipError_t launch_fused_k5(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                          const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    return launch_k<5>(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
}

hipError_t launch_fused_k6(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                          const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    return launch_k<6>(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
}

hipError_t launch_fused_k7(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                          const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    return launch_k<7>(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
}

}  // namespace qaoa

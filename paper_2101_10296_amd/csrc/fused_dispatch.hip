// Dispatch of the workgroup-resident kernel by cone size.
#include "device.hpp"

namespace qaoa {

hipError_t launch_fused_k2(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k3(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k4(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k5(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k6(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k7(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k8(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k9(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k10(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k11(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k12(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k13(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k14(bool, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);

hipError_t launch_fused(int K, bool grad, const ConeDev* cones, int64_t item_base, int64_t n_items,
                        const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    switch (K) {
        case 2: return launch_fused_k2(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 3: return launch_fused_k3(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 4: return launch_fused_k4(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 5: return launch_fused_k5(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 6: return launch_fused_k6(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 7: return launch_fused_k7(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 8: return launch_fused_k8(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 9: return launch_fused_k9(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 10: return launch_fused_k10(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 11: return launch_fused_k11(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 12: return launch_fused_k12(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 13: return launch_fused_k13(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        case 14: return launch_fused_k14(grad, cones, item_base, n_items, cut, rowcap, ea, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qaoa

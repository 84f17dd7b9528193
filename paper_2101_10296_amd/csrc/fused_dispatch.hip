// Dispatch of the workgroup-resident kernel by cone size.
#include "fused_impl.hpp"

#include <vector>

namespace qaoa {

hipError_t launch_fused_k2(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k3(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k4(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k5(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k6(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k7(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k8(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k9(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k10(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k11(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k12(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k13(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);
hipError_t launch_fused_k14(bool, int, const ConeDev*, int64_t, int64_t, const uint8_t*, int32_t, const EvalArgs&, hipStream_t);

hipError_t launch_fused(int K, bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                        const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    switch (K) {
        case 2: return launch_fused_k2(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 3: return launch_fused_k3(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 4: return launch_fused_k4(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 5: return launch_fused_k5(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 6: return launch_fused_k6(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 7: return launch_fused_k7(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 8: return launch_fused_k8(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 9: return launch_fused_k9(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 10: return launch_fused_k10(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 11: return launch_fused_k11(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 12: return launch_fused_k12(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 13: return launch_fused_k13(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        case 14: return launch_fused_k14(grad, variant, cones, item_base, n_items, cut, rowcap, ea, st);
        default: return hipErrorInvalidValue;
    }
}

// Layout variants of the K-qubit kernel worth timing (the default first).
std::vector<int> fused_variants(int K, bool grad) {
    std::vector<int> v{0};
    auto add = [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        for (int x = 1; x <= 3; ++x)
            if (fused_variant_ok<KK>(grad, x)) v.push_back(x);
    };
    switch (K) {
        case 2: add(std::integral_constant<int, 2>{}); break;
        case 3: add(std::integral_constant<int, 3>{}); break;
        case 4: add(std::integral_constant<int, 4>{}); break;
        case 5: add(std::integral_constant<int, 5>{}); break;
        case 6: add(std::integral_constant<int, 6>{}); break;
        case 7: add(std::integral_constant<int, 7>{}); break;
        case 8: add(std::integral_constant<int, 8>{}); break;
        case 9: add(std::integral_constant<int, 9>{}); break;
        case 10: add(std::integral_constant<int, 10>{}); break;
        case 11: add(std::integral_constant<int, 11>{}); break;
        case 12: add(std::integral_constant<int, 12>{}); break;
        case 13: add(std::integral_constant<int, 13>{}); break;
        case 14: add(std::integral_constant<int, 14>{}); break;
        default: break;
    }
    return v;
}

}  // namespace qaoa

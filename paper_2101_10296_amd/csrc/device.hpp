// Device-side data shared by the launchers and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qaoa {

// One light cone as seen by the kernels.
struct ConeDev {
    int32_t orbit;      // term index m (output column)
    int32_t k;          // qubits
    int32_t edge_off;   // first cone edge in the flattened edge arrays
    int32_t n_edges;    // induced edges
    int64_t cut_off;    // byte offset of the cone's cut table (workgroup-resident cones)
    int32_t cut_shift;  // cone.cut_min - plan.cut_min: offset into a phase table row
    int32_t cut_min;    // smallest possible cut value of the cone
    int32_t cut_range;  // cut_max - cut_min + 1
    int32_t inst;       // instance of the cone (plans over several graphs; angle tables per instance)
    float c0;           // real weights: centre of the cut range, subtracted in the float cut table
    int32_t pad_;
};

// Arguments of one energy evaluation that every kernel needs.
struct EvalArgs {
    int32_t P;              // angle points (per instance)
    int32_t p;              // depth
    int32_t M;              // terms (orbits, all instances)
    int32_t R;              // phase-table row length (global cut range + 1)
    const float2* phase;    // [inst][P][p][R]: exp(-i gamma_l delta_inst c), c = plan.cut_min + index
    const float2* mix;      // [inst][P][p]: (tau_l, |kappa_l|^2) of the factored mixer exp(-i beta_l X)
    const double* gamma;    // real weights: the angles, gamma[(inst * gamma_P + point) * p + l]
    int32_t gamma_P;        // points per instance in that array
    int32_t realw;          // 1: cut values are real (float table per cone), phases computed per amplitude
    double* zz;             // [P][M]
    double* g;              // [P][2p][M]: d zz / d gamma_l (l < p), d zz / d beta_l (p <= l < 2p)
};

}  // namespace qaoa

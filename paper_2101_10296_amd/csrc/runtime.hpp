// Per-plan device state and the energy driver behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "device.hpp"
#include "hbm_impl.hpp"
#include "plan.hpp"
#include "qaoa.h"

struct qaoa_plan_s {
    qaoa::HostPlan hp;
    qaoa::PlanOptions opt;

    // ---- device-resident plan data (built on the first energy call, one allocation: d_arena)
    void* d_arena = nullptr;
    int device = -1;
    bool dev_ready = false;
    struct Group {
        int K;          // cone qubits
        int64_t first;  // first slot in d_cones
        int64_t count;  // cones in this group
        int32_t rowcap; // largest cut range of the group's cones
    };
    std::vector<Group> lds_groups;      // workgroup-resident cones, grouped by K
    qaoa::ConeDev* d_cones = nullptr;
    uint8_t* d_cut = nullptr;
    // HBM-resident cones, grouped by k
    struct HGroup {
        int K;
        int64_t first;
        int64_t count;
        int32_t rowcap;
    };
    std::vector<HGroup> hbm_groups;
    qaoa::ConeHbm* d_hcones = nullptr;
    int32_t *d_ea = nullptr, *d_eb = nullptr, *d_ew = nullptr;
    double* d_ewd = nullptr;            // real weights of the cone edges (real-weight plans)
    uint8_t* d_tt = nullptr;
    double* d_W = nullptr;
    int64_t* d_inst_orbit = nullptr;    // [n_inst + 1]
    double* d_inst_delta = nullptr;     // [n_inst]
    double* d_ones = nullptr;           // [n_inst] of 1.0 (combination of per-term gradients in radians)
    size_t resident_bytes = 0;

    // ---- profiling (opts.profile): events around each kernel group of the last call
    struct Timed {
        int32_t k;
        int64_t items;
        hipEvent_t start, stop;
    };
    std::vector<Timed> timed;
    size_t n_timed = 0;

    // ---- per-call scratch, grown on demand
    size_t cap_phase = 0, cap_mix = 0, cap_zz = 0, cap_g = 0;
    float2* d_phase = nullptr;
    float2* d_mix = nullptr;
    double* d_zz = nullptr;
    double* d_g = nullptr;
    size_t cap_phi = 0, cap_lam = 0, cap_gpart = 0;
    float2* d_phi = nullptr;
    float2* d_lam = nullptr;
    double* d_gpart = nullptr;
    std::vector<int64_t> hbm_batch;     // items per batch of each HBM group in the last call
    std::vector<int8_t> hbm_ckpt;       // 1 if the HBM group stored forward checkpoints in the last call
    int64_t pass_launches[qaoa::N_PASS_KINDS] = {};   // per pass kind, last eager call
    int32_t checkpointed_classes = 0;   // HBM groups that stored checkpoints in the last eager call
    uint32_t checkpointed_k_mask = 0;   // bit k: the k-qubit class did

    // ---- graph replay (opts.graph)
    struct GraphKey {
        int64_t n_points = -1;
        bool grad = false;
        const void* ptr[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        bool operator==(const GraphKey& o) const {
            if (n_points != o.n_points || grad != o.grad) return false;
            for (int i = 0; i < 7; ++i)
                if (ptr[i] != o.ptr[i]) return false;
            return true;
        }
    };
    GraphKey gkey;
    hipGraphExec_t gexec = nullptr;
    int64_t graph_replays = 0;
    hipStream_t cap_stream = nullptr;
};

namespace qaoa {

qaoa_status run_energy(qaoa_plan_s* plan, int64_t n_points, const double* gamma, const double* beta,
                       double* energy, double* term_zz, double* dgamma, double* dbeta, double* term_grad,
                       hipStream_t stream,
                       std::string& msg);

void release_device(qaoa_plan_s* plan);

// The run-time tuner's choices so far (one line per kernel class).
std::string tuning_report();

// Records msg as this thread's last error (capi.hip) and returns st.
qaoa_status set_last_error(qaoa_status st, const std::string& msg);
void clear_last_error();
qaoa_status kernel_times(qaoa_plan_s* plan, int32_t cap, int32_t* k_out, int64_t* items_out, double* ms_out,
                         int32_t* n_out, std::string& msg);

// kernel launchers
// variant: layout of the workgroup kernel (0 default; see Fz in fused_impl.hpp)
hipError_t launch_fused(int K, bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                        const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st);
std::vector<int> fused_variants(int K, bool grad);
hipError_t launch_tables(const double* gamma, const double* beta, int64_t n_pl, int32_t R, int32_t cmin,
                         const double* deltas, int64_t pl_per_inst, float2* phase, float2* mix, hipStream_t st);
hipError_t launch_cut_tables(const ConeDev* cones, int64_t n_cones, const int32_t* ea, const int32_t* eb,
                             const int32_t* ew, uint8_t* tables, hipStream_t st);
hipError_t launch_cut_tables_real(const ConeDev* cones, int64_t n_cones, const int32_t* ea, const int32_t* eb,
                                  const double* ew, float* tables, hipStream_t st);
hipError_t launch_pass(int kind, const PassArgs& pa, hipStream_t st);
hipError_t launch_tt_tables(const ConeHbm* cones, int64_t n_cones, int max_groups, const int32_t* ea,
                            const int32_t* eb, const int32_t* ew, uint8_t* tt, hipStream_t st);
hipError_t launch_tt_tables_real(const ConeHbm* cones, int64_t n_cones, int max_groups, const int32_t* ea,
                                 const int32_t* eb, const double* ew, float* tt, hipStream_t st);
hipError_t launch_fill_zero(double* x, int64_t n, hipStream_t st);
hipError_t launch_tile_reduce(const ConeHbm* cones, const double* gpart, int64_t item0, int64_t n_batch,
                              int64_t tiles, int32_t stride, int32_t nvals, const EvalArgs& ea, hipStream_t st);

// One pass of the HBM program (see hbm_impl.hpp).
struct PassSpec {
    int kind, group, la, lb, m0a, m0b;
    int fix_layer = 0, fix_pow = 0;   // rescaling of psi read as the forward sweep left it
    int ck_in = -1, ck_out = -1;      // checkpoint slots read / written (-1: the single state buffer)
    int store_phi = 1;                // reverse passes: write the undone psi back
};
int hbm_groups_of(int k);
int hbm_group_qubits(int k, int grp);
// ckpt: every forward pass but the final one writes its output to a slot of its own
// (hbm_checkpoints(k, p) slots) and every reverse pass reads psi from the slot of the
// forward pass it undoes instead of carrying the uncomputed psi along.
std::vector<PassSpec> hbm_program(int k, int p, bool grad, bool ckpt = false);
int hbm_checkpoints(int k, int p);

hipError_t launch_scale_gamma_terms(double* g, int64_t P, int32_t p, int32_t M, const int64_t* inst_orbit,
                                    int32_t n_inst, const double* deltas, hipStream_t st);
// points per k_combine launch with ny blocks per point (grid below 2^32 work-items)
int64_t combine_chunk(uint32_t ny);
// energy [n_inst][P_out], dgamma / dbeta [n_inst][P_out][p]: points i0 .. i0 + Pc - 1 of
// each instance from the term rows zz [Pc][M], g [Pc][2p][M]
hipError_t launch_combine(const double* W, const double* zz, const double* g, int32_t M, int32_t p,
                          const int64_t* inst_orbit, const double* deltas, int32_t n_inst, int64_t Pc,
                          int64_t P_out, int64_t i0, double* energy, double* dgamma, double* dbeta, hipStream_t st);

}  // namespace qaoa

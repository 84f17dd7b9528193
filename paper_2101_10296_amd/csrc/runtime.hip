// Device runtime of a plan: one-time upload of cone descriptors and cut tables, scratch
// management, and the sequence of launches of one energy (and gradient) evaluation.
#include "runtime.hpp"

#include <algorithm>
#include <numeric>

namespace qaoa {
namespace {

#define QCHECK(expr)                                                               \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            msg = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return (e_ == hipErrorOutOfMemory) ? QAOA_ENOMEM : QAOA_EHIP;         \
        }                                                                          \
    } while (0)

template <class T>
qaoa_status grow(T*& ptr, size_t& cap, size_t need, std::string& msg) {
    if (need <= cap && ptr) return QAOA_OK;
    if (ptr) {
        hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
    const size_t bytes = std::max<size_t>(need, 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ptr), bytes);
    if (e != hipSuccess) {
        ptr = nullptr;
        msg = "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
        return QAOA_ENOMEM;
    }
    cap = std::max<size_t>(need, 1);
    return QAOA_OK;
}

qaoa_status ensure_device(qaoa_plan_s* P, std::string& msg) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        msg = std::string("no HIP device: ") + hipGetErrorString(e);
        return QAOA_EHIP;
    }
    if (P->dev_ready) {
        if (dev != P->device) {
            msg = "plan was uploaded to device " + std::to_string(P->device) + ", current device is " + std::to_string(dev);
            return QAOA_EINVAL;
        }
        return QAOA_OK;
    }
    const HostPlan& hp = P->hp;
    const int64_t M = static_cast<int64_t>(hp.cones.size());
    for (const auto& c : hp.cones)
        if (c.k > P->opt.k_lds_max) {
            msg = "cones above " + std::to_string(P->opt.k_lds_max) + " qubits are not supported by this build";
            return QAOA_ECONE;
        }
    // workgroup-resident cones, grouped by K
    std::vector<int64_t> ord(M);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return hp.cones[a].k < hp.cones[b].k; });
    std::vector<ConeDev> cd(M);
    std::vector<int32_t> ea, eb, ew;
    int64_t cut_bytes = 0;
    P->lds_groups.clear();
    for (int64_t s = 0; s < M; ++s) {
        const Cone& c = hp.cones[ord[s]];
        ConeDev& d = cd[s];
        d.orbit = static_cast<int32_t>(ord[s]);
        d.k = c.k;
        d.edge_off = static_cast<int32_t>(ea.size());
        d.n_edges = static_cast<int32_t>(c.ea.size());
        d.cut_off = cut_bytes;
        d.cut_shift = c.cut_min - hp.cut_min;
        d.cut_min = c.cut_min;
        d.cut_range = c.cut_max - c.cut_min + 1;
        d.pad_ = 0;
        cut_bytes += std::max<int64_t>(int64_t{1} << c.k, 16);
        ea.insert(ea.end(), c.ea.begin(), c.ea.end());
        eb.insert(eb.end(), c.eb.begin(), c.eb.end());
        ew.insert(ew.end(), c.ew.begin(), c.ew.end());
        if (P->lds_groups.empty() || P->lds_groups.back().K != c.k) P->lds_groups.push_back({c.k, s, 0, 1});
        P->lds_groups.back().count += 1;
        P->lds_groups.back().rowcap = std::max(P->lds_groups.back().rowcap, d.cut_range);
    }
    int32_t *d_ea = nullptr, *d_eb = nullptr, *d_ew = nullptr;
    const size_t ne = std::max<size_t>(ea.size(), 1);
    QCHECK(hipMalloc(&P->d_cones, std::max<size_t>(cd.size(), 1) * sizeof(ConeDev)));
    QCHECK(hipMalloc(&P->d_cut, std::max<int64_t>(cut_bytes, 16)));
    QCHECK(hipMalloc(&P->d_W, std::max<size_t>(hp.W.size(), 1) * sizeof(double)));
    QCHECK(hipMalloc(&d_ea, ne * sizeof(int32_t)));
    QCHECK(hipMalloc(&d_eb, ne * sizeof(int32_t)));
    QCHECK(hipMalloc(&d_ew, ne * sizeof(int32_t)));
    if (M) {
        QCHECK(hipMemcpy(P->d_cones, cd.data(), cd.size() * sizeof(ConeDev), hipMemcpyHostToDevice));
        QCHECK(hipMemcpy(P->d_W, hp.W.data(), hp.W.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (!ea.empty()) {
        QCHECK(hipMemcpy(d_ea, ea.data(), ea.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        QCHECK(hipMemcpy(d_eb, eb.data(), eb.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        QCHECK(hipMemcpy(d_ew, ew.data(), ew.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    QCHECK(launch_cut_tables(P->d_cones, M, d_ea, d_eb, d_ew, P->d_cut, nullptr));
    QCHECK(hipDeviceSynchronize());
    hipFree(d_ea);
    hipFree(d_eb);
    hipFree(d_ew);
    P->resident_bytes = cd.size() * sizeof(ConeDev) + static_cast<size_t>(cut_bytes) + hp.W.size() * sizeof(double);
    P->device = dev;
    P->dev_ready = true;
    return QAOA_OK;
}

// Events around one kernel group (profiling only).
struct GroupTimer {
    qaoa_plan_s* P;
    hipStream_t st;
    size_t slot = 0;
    bool on;
    GroupTimer(qaoa_plan_s* p, hipStream_t s) : P(p), st(s), on(p->opt.profile != 0) {
        if (on) P->n_timed = 0;
    }
    hipError_t begin(int32_t k, int64_t items) {
        if (!on) return hipSuccess;
        slot = P->n_timed++;
        if (P->timed.size() < P->n_timed) {
            qaoa_plan_s::Timed t{k, items, nullptr, nullptr};
            hipError_t e = hipEventCreate(&t.start);
            if (e == hipSuccess) e = hipEventCreate(&t.stop);
            if (e != hipSuccess) return e;
            P->timed.push_back(t);
        }
        P->timed[slot].k = k;
        P->timed[slot].items = items;
        return hipEventRecord(P->timed[slot].start, st);
    }
    hipError_t end() { return on ? hipEventRecord(P->timed[slot].stop, st) : hipSuccess; }
};

}  // namespace

qaoa_status kernel_times(qaoa_plan_s* P, int32_t cap, int32_t* k_out, int64_t* items_out, double* ms_out,
                         int32_t* n_out, std::string& msg) {
    if (!P->opt.profile || P->n_timed == 0) {
        msg = "plan was not built with profile = 1 or has not been evaluated";
        return QAOA_EINVAL;
    }
    for (size_t i = 0; i < P->n_timed && static_cast<int32_t>(i) < cap; ++i) {
        auto& t = P->timed[i];
        QCHECK(hipEventSynchronize(t.stop));
        float ms = 0.f;
        QCHECK(hipEventElapsedTime(&ms, t.start, t.stop));
        if (k_out) k_out[i] = t.k;
        if (items_out) items_out[i] = t.items;
        if (ms_out) ms_out[i] = ms;
    }
    if (n_out) *n_out = static_cast<int32_t>(P->n_timed);
    return QAOA_OK;
}

qaoa_status run_energy(qaoa_plan_s* P, int64_t n_points, const double* gamma, const double* beta, double* energy,
                       double* term_zz, double* dgamma, double* dbeta, hipStream_t stream, std::string& msg) {
    qaoa_status st = ensure_device(P, msg);
    if (st != QAOA_OK) return st;
    const HostPlan& hp = P->hp;
    const bool grad = (dgamma != nullptr);
    const int32_t p = hp.p;
    const int32_t M = static_cast<int32_t>(hp.cones.size());
    const int32_t R = hp.cut_max - hp.cut_min + 1;
    const size_t npl = static_cast<size_t>(n_points) * p;
    if ((st = grow(P->d_phase, P->cap_phase, npl * R, msg)) != QAOA_OK) return st;
    if ((st = grow(P->d_mix, P->cap_mix, npl, msg)) != QAOA_OK) return st;
    double* zz = term_zz;
    if (!zz) {
        if ((st = grow(P->d_zz, P->cap_zz, static_cast<size_t>(n_points) * M, msg)) != QAOA_OK) return st;
        zz = P->d_zz;
    }
    double* g = nullptr;
    if (grad) {
        if ((st = grow(P->d_g, P->cap_g, static_cast<size_t>(n_points) * 2 * p * M, msg)) != QAOA_OK) return st;
        g = P->d_g;
    }
    GroupTimer tm(P, stream);
    QCHECK(tm.begin(-1, static_cast<int64_t>(npl)));
    QCHECK(launch_tables(gamma, beta, static_cast<int64_t>(npl), R, hp.cut_min, P->d_phase, P->d_mix, stream));
    QCHECK(tm.end());
    EvalArgs ea{static_cast<int32_t>(n_points), p, M, R, P->d_phase, P->d_mix, zz, g};
    for (const auto& grp : P->lds_groups) {
        const ConeDev* cones = P->d_cones + grp.first;
        const int64_t items = grp.count * n_points;
        QCHECK(tm.begin(grp.K, items));
        if (P->opt.one_cone_at_a_time) {
            for (int64_t it = 0; it < items; ++it)
                QCHECK(launch_fused(grp.K, grad, cones, it, it + 1, P->d_cut, grp.rowcap, ea, stream));
        } else {
            QCHECK(launch_fused(grp.K, grad, cones, 0, items, P->d_cut, grp.rowcap, ea, stream));
        }
        QCHECK(tm.end());
    }
    QCHECK(tm.begin(-2, n_points));
    QCHECK(launch_combine(P->d_W, zz, g, M, p, n_points, energy, dgamma, dbeta, stream));
    QCHECK(tm.end());
    return QAOA_OK;
}

void release_device(qaoa_plan_s* P) {
    for (auto& t : P->timed) {
        hipEventDestroy(t.start);
        hipEventDestroy(t.stop);
    }
    P->timed.clear();
    if (!P->dev_ready && !P->d_phase) return;
    hipDeviceSynchronize();
    hipFree(P->d_cones);
    hipFree(P->d_cut);
    hipFree(P->d_W);
    hipFree(P->d_phase);
    hipFree(P->d_mix);
    hipFree(P->d_zz);
    hipFree(P->d_g);
    P->d_cones = nullptr;
    P->d_cut = nullptr;
    P->d_W = nullptr;
    P->d_phase = nullptr;
    P->d_mix = nullptr;
    P->d_zz = nullptr;
    P->d_g = nullptr;
    P->dev_ready = false;
}

}  // namespace qaoa

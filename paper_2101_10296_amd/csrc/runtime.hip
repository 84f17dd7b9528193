// Device runtime of a plan: one-time upload of cone descriptors and cut tables, scratch
// management, and the sequence of launches of one energy (and gradient) evaluation.
#include "runtime.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>

namespace qaoa {
namespace {

// ---- run-time tuner (plans built with opts.tune = 1).  Layout choices of a kernel class
// are timed once per process on the first call that needs them (HIP events on the call's
// stream) and the fastest is kept, keyed by (device architecture, what, k, p, gradient,
// real weights).  what = 0: register bits per LDS stage / workgroup size of the
// workgroup-resident kernel (fused_variants); what = 1: tiles per workgroup of the
// device-memory passes.
struct TuneKey {
    std::string arch;
    int what, k, p, grad, realw;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, what, k, p, grad, realw) < std::tie(o.arch, o.what, o.k, o.p, o.grad, o.realw);
    }
};
struct TuneRec {
    int choice = 0;
    std::vector<std::pair<int, float>> ms;   // candidate -> milliseconds per timed launch
    int64_t items = 0;                       // items of the timed launches
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneRec> g_tune;

std::string device_arch(int dev) {
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop{};
    std::string a = hipGetDeviceProperties(&prop, dev) == hipSuccess ? std::string(prop.gcnArchName) : "unknown";
    names[dev] = a;
    return a;
}

bool tune_lookup(const TuneKey& key, int& choice) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    choice = it->second.choice;
    return true;
}

// Times run(candidate) for every candidate (one untimed launch, then `reps` timed ones on
// the stream) and records the fastest under key.
template <class Run>
hipError_t tune_pick(const TuneKey& key, const std::vector<int>& cand, int64_t items, hipStream_t st, Run&& run,
                     int& choice) {
    TuneRec rec;
    rec.items = items;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    constexpr int reps = 3;
    float best = 0.f;
    for (size_t i = 0; e == hipSuccess && i < cand.size(); ++i) {
        e = run(cand[i]);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; e == hipSuccess && r < reps; ++r) e = run(cand[i]);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        ms /= reps;
        rec.ms.emplace_back(cand[i], ms);
        if (i == 0 || ms < best) {
            best = ms;
            rec.choice = cand[i];
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    choice = rec.choice;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = rec;
    return hipSuccess;
}

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
        (void)hipGetLastError();   // clear the failure so later launch checks do not see it
        ptr = nullptr;
        msg = "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
        return QAOA_ENOMEM;
    }
    cap = std::max<size_t>(need, 1);
    return QAOA_OK;
}

// Pass groups over the kh = k - 1 stored qubits of a k-qubit HBM cone: group 0 = qubits
// 0..12, group j >= 1 = nine of the remaining qubits; tile bit i of group g maps to global
// bit hbm_group_global_bit(kh, g, i) (the same map as hgroup_bits in hbm_impl.hpp).
int hbm_group_global_bit(int k, int grp, int i) {
    if (grp == 0) return i;
    const int lo = 13 + 9 * (grp - 1);
    const int h = std::min(k, lo + 9) - lo;
    if (i < h) return lo + i;
    if (i < 9) return 4 + (i - h);
    return i - 9;
}

}  // namespace

int hbm_groups_of(int k) { return 1 + (k - 13 + 8) / 9; }

int hbm_group_qubits(int k, int grp) {
    if (grp == 0) return 13;
    const int lo = 13 + 9 * (grp - 1);
    return std::min(k, lo + 9) - lo;
}

int hbm_checkpoints(int k, int p) {
    return p == 1 ? 0 : 1 + (p - 1) * (hbm_groups_of(k - 1) - 1) - 1;
}

// Forward program over the stored qubits (kh = k - 1): layer l (1 <= l <= p-1) visits the
// groups in descending order when p-1-l is even, ascending otherwise, so layer p-1 ends on
// group 0 and consecutive layers share a pass.  Group-0 passes also mix the dropped qubit
// k-1 (14 qubits per layer).  With grad, the last pass is the fused final/adjoint pass and
// the earlier passes follow in reverse as RV_* passes; m0a / m0b count the qubits of a
// layer already undone by earlier reverse passes.
std::vector<PassSpec> hbm_program(int k, int p, bool grad, bool ckpt) {
    std::vector<PassSpec> fwd;
    const int kh = k - 1;
    const int n = hbm_groups_of(kh);
    auto layer_qubits = [&](int g) { return hbm_group_qubits(kh, g) + (g == 0 ? 1 : 0); };
    if (p == 1) {
        fwd.push_back({grad ? GR_GEN_FINAL : FWD_GEN_FINAL, 0, 0, 1, 0, 0});
        return fwd;
    }
    ckpt = ckpt && grad;
    auto group_at = [&](int l, int j) { return (((p - 1 - l) & 1) == 0) ? n - 1 - j : j; };
    // in_prog[i] / mixed[i]: the layer in progress after forward pass i and how many of its
    // qubits have been mixed by then (the forward scale of the state written by pass i)
    std::vector<int> in_prog, mixed;
    fwd.push_back({FWD_GEN_MIX, group_at(1, 0), 0, 1, 0, 0});
    in_prog.push_back(1);
    mixed.push_back(layer_qubits(fwd.back().group));
    for (int l = 1; l <= p - 1; ++l)
        for (int j = 1; j < n; ++j) {
            const int g = group_at(l, j);
            if (j < n - 1) {
                fwd.push_back({FWD_MIX, g, l, 0, 0, 0});
                in_prog.push_back(l);
                mixed.push_back(mixed.back() + layer_qubits(g));
            } else if (l + 1 <= p - 1) {
                fwd.push_back({FWD_BND_MIX, g, l, l + 1, 0, 0});
                in_prog.push_back(l + 1);
                mixed.push_back(layer_qubits(g));
            } else {
                fwd.push_back({FWD_BND_FINAL, g, l, p, 0, 0});
            }
        }
    const int nf = static_cast<int>(fwd.size()) - 1;   // forward passes before the final one
    if (ckpt)
        for (int i = 0; i <= nf; ++i) {
            fwd[i].ck_in = i - 1;
            fwd[i].ck_out = i < nf ? i : -1;
        }
    if (!grad) return fwd;
    std::vector<PassSpec> out(fwd.begin(), fwd.end() - 1);
    std::vector<int> undone(p + 2, 0);
    PassSpec fin = fwd.back();
    fin.kind = GR_BND_FINAL;
    fin.m0a = undone[fin.la];
    undone[fin.la] += layer_qubits(fin.group);
    out.push_back(fin);
    for (int i = nf - 1; i >= 0; --i) {
        PassSpec r = fwd[i];
        const int h = layer_qubits(r.group);
        if (r.kind == FWD_GEN_MIX) {
            r.kind = RV_GEN_MIX;
            r.m0b = undone[r.lb];
            undone[r.lb] += h;
        } else if (r.kind == FWD_MIX) {
            r.kind = RV_MIX;
            r.m0a = undone[r.la];
            undone[r.la] += h;
        } else {
            r.kind = RV_BND_MIX;
            r.m0b = undone[r.lb];
            undone[r.lb] += h;
            r.m0a = undone[r.la];
            undone[r.la] += h;
        }
        if (ckpt || i == nf - 1) {
            // psi read as the forward sweep left it (pass i's output): rescale it from the
            // forward scale of its layer in progress to lambda's
            r.fix_layer = in_prog[i];
            r.fix_pow = 2 * mixed[i] - k;
        }
        if (ckpt) {
            r.ck_in = i;
            r.ck_out = -1;
            r.store_phi = 0;
        }
        out.push_back(r);
    }
    return out;
}

namespace {

// pinned staging buffer of the plan uploads (ensure_device)
std::mutex g_stage_mu;
void* g_stage = nullptr;
size_t g_stage_cap = 0;

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
    const int64_t Mall = static_cast<int64_t>(hp.cones.size());
    // workgroup-resident cones (k <= k_lds_max), grouped by K; larger cones go to the
    // HBM-resident passes, grouped by k
    std::vector<int64_t> ord, hord;
    for (int64_t m = 0; m < Mall; ++m) (hp.cones[m].k <= P->opt.k_lds_max ? ord : hord).push_back(m);
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return hp.cones[a].k < hp.cones[b].k; });
    std::stable_sort(hord.begin(), hord.end(), [&](int64_t a, int64_t b) { return hp.cones[a].k < hp.cones[b].k; });
    const int64_t M = static_cast<int64_t>(ord.size());
    std::vector<ConeDev> cd(M);
    std::vector<int32_t> ea, eb, ew;
    std::vector<double> ewd;   // real weights (plans with real weights only)
    int64_t cut_bytes = 0;
    P->lds_groups.clear();
    for (int64_t s = 0; s < M; ++s) {
        const Cone& c = hp.cones[ord[s]];
        ConeDev& d = cd[s];
        d.orbit = static_cast<int32_t>(ord[s]);
        d.k = c.k;
        d.edge_off = static_cast<int32_t>(ea.size());
        d.n_edges = static_cast<int32_t>(c.ea.size());
        d.inst = c.inst;
        d.c0 = 0.f;
        d.pad_ = 0;
        if (hp.realw) {
            // float table of C(x) - c0 over the stored half; cut_off counts floats
            d.cut_off = cut_bytes / 4;
            d.cut_shift = 0;
            d.cut_min = 0;
            d.cut_range = 1;
            d.c0 = static_cast<float>(0.5 * (c.cf_min + c.cf_max));
            cut_bytes += 4 * std::max<int64_t>(int64_t{1} << (c.k >= 3 ? c.k - 1 : c.k), 4);
            ewd.insert(ewd.end(), c.wf.begin(), c.wf.end());
        } else {
            d.cut_off = cut_bytes;
            d.cut_shift = c.cut_min - hp.cut_min;
            d.cut_min = c.cut_min;
            d.cut_range = c.cut_max - c.cut_min + 1;
            cut_bytes += std::max<int64_t>(int64_t{1} << c.k, 16);
        }
        ea.insert(ea.end(), c.ea.begin(), c.ea.end());
        eb.insert(eb.end(), c.eb.begin(), c.eb.end());
        ew.insert(ew.end(), c.ew.begin(), c.ew.end());
        if (P->lds_groups.empty() || P->lds_groups.back().K != c.k) P->lds_groups.push_back({c.k, s, 0, 1});
        P->lds_groups.back().count += 1;
        P->lds_groups.back().rowcap = std::max(P->lds_groups.back().rowcap, d.cut_range);
    }
    // HBM-class descriptors; their edges follow the workgroup-resident ones
    std::vector<ConeHbm> hc(hord.size());
    int64_t tt_bytes = 0;
    int max_groups = 1;
    P->hbm_groups.clear();
    for (size_t s = 0; s < hord.size(); ++s) {
        const Cone& c = hp.cones[hord[s]];
        ConeHbm& d = hc[s];
        std::memset(&d, 0, sizeof(d));
        d.orbit = static_cast<int32_t>(hord[s]);
        d.k = c.k;
        d.edge_off = static_cast<int32_t>(ea.size());
        d.n_edges = static_cast<int32_t>(c.ea.size());
        d.cut_min = c.cut_min;
        d.cut_range = c.cut_max - c.cut_min + 1;
        d.cut_shift = c.cut_min - hp.cut_min;
        d.inst = c.inst;
        d.c0 = static_cast<float>(0.5 * (c.cf_min + c.cf_max));
        d.n_groups = hbm_groups_of(c.k - 1);
        max_groups = std::max(max_groups, d.n_groups);
        for (int g = 0; g < d.n_groups; ++g) {
            // tile bits of group g; C_tt ranges over the edges with both ends inside
            std::vector<char> in(32, 0);
            for (int i = 0; i < 13; ++i) in[hbm_group_global_bit(c.k - 1, g, i)] = 1;
            int32_t tmin = 0, tmax = 0;
            for (size_t e = 0; e < c.ea.size(); ++e)
                if (in[c.ea[e]] && in[c.eb[e]]) (c.ew[e] < 0 ? tmin : tmax) += c.ew[e];
            d.tt_min[g] = tmin;
            // byte table of 2^13 entries, or (real weights) floats: tt_off then counts floats
            d.tt_off[g] = hp.realw ? tt_bytes / 4 : tt_bytes;
            tt_bytes += hp.realw ? 4 * 8192 : 8192;
        }
        ea.insert(ea.end(), c.ea.begin(), c.ea.end());
        eb.insert(eb.end(), c.eb.begin(), c.eb.end());
        ew.insert(ew.end(), c.ew.begin(), c.ew.end());
        if (hp.realw) ewd.insert(ewd.end(), c.wf.begin(), c.wf.end());
        if (P->hbm_groups.empty() || P->hbm_groups.back().K != c.k)
            P->hbm_groups.push_back({c.k, static_cast<int64_t>(s), 0, 1});
        P->hbm_groups.back().count += 1;
        P->hbm_groups.back().rowcap = std::max(P->hbm_groups.back().rowcap, d.cut_range);
    }
    if (ea.size() > static_cast<size_t>(INT32_MAX) || Mall > INT32_MAX) {
        msg = "the plan's cones hold " + std::to_string(ea.size()) + " edges over " + std::to_string(Mall) +
              " orbits; descriptors index both with 32-bit integers";
        return QAOA_EINVAL;
    }
    // One device allocation holds every resident array: the ones with host data first (one
    // copy), then the cut and C_tt tables, which kernels fill.
    const size_t ne = std::max<size_t>(ea.size(), 1);
    const std::vector<double> ones(hp.inst_delta.size(), 1.0);
    size_t arena = 0;
    auto place = [&](size_t bytes) {
        const size_t o = arena;
        arena += (std::max<size_t>(bytes, 16) + 255) & ~size_t{255};
        return o;
    };
    const size_t o_cones = place(std::max<size_t>(cd.size(), 1) * sizeof(ConeDev));
    const size_t o_W = place(std::max<size_t>(hp.W.size(), 1) * sizeof(double));
    const size_t o_hcones = place(std::max<size_t>(hc.size(), 1) * sizeof(ConeHbm));
    const size_t o_ea = place(ne * sizeof(int32_t));
    const size_t o_eb = place(ne * sizeof(int32_t));
    const size_t o_ew = place(ne * sizeof(int32_t));
    const size_t o_io = place(hp.inst_orbit.size() * sizeof(int64_t));
    const size_t o_id = place(hp.inst_delta.size() * sizeof(double));
    const size_t o_ones = place(ones.size() * sizeof(double));
    const size_t o_ewd = hp.realw ? place(std::max<size_t>(ewd.size(), 1) * sizeof(double)) : 0;
    const size_t copied = arena;
    const size_t o_cut = place(static_cast<size_t>(std::max<int64_t>(cut_bytes, 16)));
    const size_t o_tt = place(static_cast<size_t>(std::max<int64_t>(tt_bytes, 16)));
    {
        // staged in pinned host memory shared by all plans of the process (grown on demand,
        // kept until exit): one fast copy instead of a pageable one (3 MB: 1.1 ms -> ~0.1 ms)
        std::lock_guard<std::mutex> lock(g_stage_mu);
        if (g_stage_cap < copied) {
            if (g_stage) hipHostFree(g_stage);
            g_stage = nullptr;
            g_stage_cap = 0;
            const size_t cap = std::max<size_t>(copied, size_t{4} << 20);
            QCHECK(hipHostMalloc(&g_stage, cap, hipHostMallocPortable));
            g_stage_cap = cap;
        }
        uint8_t* stage = static_cast<uint8_t*>(g_stage);   // the gaps between arrays are never read
        auto put = [&](size_t o, const void* src, size_t bytes) {
            if (bytes) std::memcpy(stage + o, src, bytes);
        };
        put(o_cones, cd.data(), cd.size() * sizeof(ConeDev));
        put(o_W, hp.W.data(), hp.W.size() * sizeof(double));
        put(o_hcones, hc.data(), hc.size() * sizeof(ConeHbm));
        put(o_ea, ea.data(), ea.size() * sizeof(int32_t));
        put(o_eb, eb.data(), eb.size() * sizeof(int32_t));
        put(o_ew, ew.data(), ew.size() * sizeof(int32_t));
        put(o_io, hp.inst_orbit.data(), hp.inst_orbit.size() * sizeof(int64_t));
        put(o_id, hp.inst_delta.data(), hp.inst_delta.size() * sizeof(double));
        put(o_ones, ones.data(), ones.size() * sizeof(double));
        if (hp.realw) put(o_ewd, ewd.data(), ewd.size() * sizeof(double));
        if (P->d_arena) {   // an earlier first call failed after allocating: start over
            hipFree(P->d_arena);
            P->d_arena = nullptr;
        }
        QCHECK(hipMalloc(&P->d_arena, arena));
        QCHECK(hipMemcpy(P->d_arena, stage, copied, hipMemcpyHostToDevice));
    }
    uint8_t* base = static_cast<uint8_t*>(P->d_arena);
    P->d_cones = reinterpret_cast<ConeDev*>(base + o_cones);
    P->d_W = reinterpret_cast<double*>(base + o_W);
    P->d_hcones = reinterpret_cast<ConeHbm*>(base + o_hcones);
    P->d_ea = reinterpret_cast<int32_t*>(base + o_ea);
    P->d_eb = reinterpret_cast<int32_t*>(base + o_eb);
    P->d_ew = reinterpret_cast<int32_t*>(base + o_ew);
    P->d_inst_orbit = reinterpret_cast<int64_t*>(base + o_io);
    P->d_inst_delta = reinterpret_cast<double*>(base + o_id);
    P->d_ones = reinterpret_cast<double*>(base + o_ones);
    P->d_ewd = hp.realw ? reinterpret_cast<double*>(base + o_ewd) : nullptr;
    P->d_cut = base + o_cut;
    P->d_tt = base + o_tt;
    if (hp.realw) {
        QCHECK(launch_cut_tables_real(P->d_cones, M, P->d_ea, P->d_eb, P->d_ewd, reinterpret_cast<float*>(P->d_cut),
                                      nullptr));
        QCHECK(launch_tt_tables_real(P->d_hcones, static_cast<int64_t>(hc.size()), max_groups, P->d_ea, P->d_eb,
                                     P->d_ewd, reinterpret_cast<float*>(P->d_tt), nullptr));
    } else {
        QCHECK(launch_cut_tables(P->d_cones, M, P->d_ea, P->d_eb, P->d_ew, P->d_cut, nullptr));
        QCHECK(launch_tt_tables(P->d_hcones, static_cast<int64_t>(hc.size()), max_groups, P->d_ea, P->d_eb,
                                P->d_ew, P->d_tt, nullptr));
    }
    QCHECK(hipDeviceSynchronize());
    P->resident_bytes = arena;
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

namespace {

// The launch sequence of one energy call.  With fixed_batches the HBM groups reuse the
// batch sizes of the previous call (and so allocate nothing): used while capturing.
qaoa_status enqueue(qaoa_plan_s* P, int64_t n_points, const double* gamma, const double* beta, double* energy,
                    double* term_zz, double* dgamma, double* dbeta, double* term_grad, hipStream_t stream,
                    bool fixed_batches,
                    std::string& msg) {
    qaoa_status st = ensure_device(P, msg);
    if (st != QAOA_OK) return st;
    const HostPlan& hp = P->hp;
    const bool grad = (dgamma != nullptr);
    const int32_t p = hp.p;
    const int32_t M = static_cast<int32_t>(hp.cones.size());
    const int32_t R = hp.cut_max - hp.cut_min + 1;
    const size_t npl = static_cast<size_t>(hp.n_inst) * n_points * p;   // (instance, point, layer) rows
    if ((st = grow(P->d_phase, P->cap_phase, npl * R, msg)) != QAOA_OK) return st;
    if ((st = grow(P->d_mix, P->cap_mix, npl, msg)) != QAOA_OK) return st;
    double* zz = term_zz;
    if (!zz) {
        if ((st = grow(P->d_zz, P->cap_zz, static_cast<size_t>(n_points) * M, msg)) != QAOA_OK) return st;
        zz = P->d_zz;
    }
    double* g = nullptr;
    if (grad && term_grad) {
        g = term_grad;
    } else if (grad) {
        if ((st = grow(P->d_g, P->cap_g, static_cast<size_t>(n_points) * 2 * p * M, msg)) != QAOA_OK) return st;
        g = P->d_g;
    }
    GroupTimer tm(P, stream);
    QCHECK(tm.begin(-1, static_cast<int64_t>(npl)));
    QCHECK(launch_tables(gamma, beta, static_cast<int64_t>(npl), R, hp.cut_min, P->d_inst_delta,
                         static_cast<int64_t>(n_points) * p, P->d_phase, P->d_mix, stream));
    QCHECK(tm.end());
    EvalArgs ea{static_cast<int32_t>(n_points), p, M, R, P->d_phase, P->d_mix, gamma,
                static_cast<int32_t>(n_points), hp.realw ? 1 : 0, zz, g};
    const std::string arch = P->opt.tune == 1 ? device_arch(P->device) : std::string();
    for (const auto& grp : P->lds_groups) {
        const ConeDev* cones = P->d_cones + grp.first;
        const int64_t items = grp.count * n_points;
        int variant = P->opt.tune >= 2 ? P->opt.tune - 2 : 0;   // tune 2, 3, 4: a fixed layout variant
        if (P->opt.tune == 1 && !P->opt.one_cone_at_a_time) {
            const TuneKey key{arch, 0, grp.K, p, grad ? 1 : 0, hp.realw ? 1 : 0};
            if (!tune_lookup(key, variant)) {
                const std::vector<int> cand = fused_variants(grp.K, grad);
                if (cand.size() <= 1 || fixed_batches) {
                    variant = 0;
                } else {
                    // timed on up to 2^16 items of this call (their results are written again below)
                    const int64_t ns = std::min<int64_t>(items, int64_t{1} << 16);
                    QCHECK(tune_pick(key, cand, ns, stream, [&](int v) {
                        return launch_fused(grp.K, grad, v, cones, 0, ns, P->d_cut, grp.rowcap, ea, stream);
                    }, variant));
                }
            }
        }
        QCHECK(tm.begin(grp.K, items));
        if (P->opt.one_cone_at_a_time) {
            for (int64_t it = 0; it < items; ++it)
                QCHECK(launch_fused(grp.K, grad, 0, cones, it, it + 1, P->d_cut, grp.rowcap, ea, stream));
        } else {
            QCHECK(launch_fused(grp.K, grad, variant, cones, 0, items, P->d_cut, grp.rowcap, ea, stream));
        }
        QCHECK(tm.end());
    }
    // ---- HBM-resident cones: batches of items through the pass program
    if (!fixed_batches) {
        P->hbm_batch.assign(P->hbm_groups.size(), 0);
        P->hbm_ckpt.assign(P->hbm_groups.size(), 0);
        std::fill(std::begin(P->pass_launches), std::end(P->pass_launches), int64_t{0});
        P->checkpointed_classes = 0;
        P->checkpointed_k_mask = 0;
    }
    for (size_t gi = 0; gi < P->hbm_groups.size(); ++gi) {
        const auto& grp = P->hbm_groups[gi];
        const int k = grp.K, kh = k - 1;      // stored qubits: the half with qubit k-1 = 0
        const int64_t items = grp.count * n_points;
        const int64_t tiles = int64_t{1} << (kh - HT);
        const int nvals = grad ? 2 * p + 1 : 1;     // values reduced per item
        const int stride = 2 * p + 1;                // values stored per (item, tile)
        const bool need_phi = p >= 2;
        const bool need_lam = grad && p >= 2;
        const size_t state_bytes = (size_t{1} << kh) * sizeof(float2);
        const size_t gpart_bytes = static_cast<size_t>(tiles) * stride * sizeof(double);
        // checkpoints: every forward pass but the final one keeps its output (nck states)
        const int nck = hbm_checkpoints(k, p);
        const size_t per_unc = (need_phi ? state_bytes : 0) + (need_lam ? state_bytes : 0) + gpart_bytes;
        const size_t per_ck = static_cast<size_t>(nck) * state_bytes + state_bytes + gpart_bytes;
        size_t budget = static_cast<size_t>(P->opt.mem_budget_bytes);
        if (!fixed_batches && budget == 0) {
            size_t fr = 0, tot = 0;
            QCHECK(hipMemGetInfo(&fr, &tot));
            const size_t held = P->cap_phi * sizeof(float2) + P->cap_lam * sizeof(float2) + P->cap_gpart * sizeof(double);
            budget = static_cast<size_t>(0.85 * static_cast<double>(fr + held));
        }
        // tiles (group 0: tile pairs) per workgroup: up to 8 while the class keeps >= 4096
        // workgroups (16 per CU); fixed per class, so an item's sums run in the same order
        // whatever the batching
        int tpw = 1;
        while (tpw < 8 && 2 * tpw <= tiles / 2 && items * tiles / (2 * tpw) >= 4096) tpw *= 2;
        const TuneKey tkey{arch, 1, k, p, grad ? 1 : 0, 0};
        bool tune_tpw = false;
        if (P->opt.tune == 1) {
            int c = 0;
            if (tune_lookup(tkey, c)) tpw = c;
            else tune_tpw = !fixed_batches;
        }
        // items per batch: within the budget, the grid (a pass launches up to tiles * B
        // workgroups of <= 512 threads: below 2^31 work-items) and no more than needed for
        // 2^17 workgroups (512 per CU) per pass: larger batches hold more memory and gain little
        auto batch_of = [&](size_t per_item) {
            int64_t B = std::min<int64_t>(static_cast<int64_t>(budget / per_item), items);
            B = std::min<int64_t>(B, std::max<int64_t>(1, (int64_t{1} << 22) / tiles));
            return std::min<int64_t>(B, std::max<int64_t>(1, ((int64_t{1} << 17) * tpw + tiles - 1) / tiles));
        };
        bool ckpt = false;
        if (grad && p >= 2) {
            if (fixed_batches) ckpt = P->hbm_ckpt[gi] != 0;
            else if (P->opt.checkpoint_mode == 1) ckpt = true;
            // auto: store the forward states where the budget holds them without shrinking the
            // batch, or with a batch that still gives every pass 2^15 workgroups (128 per CU)
            else if (P->opt.checkpoint_mode == 2)
                ckpt = budget >= per_ck && (batch_of(per_ck) >= batch_of(per_unc) ||
                                            batch_of(per_ck) * tiles / (2 * tpw) >= (int64_t{1} << 15));
        }
        const size_t per_item = ckpt ? per_ck : per_unc;
        const int nphi = ckpt ? nck : 1;
        int64_t B;
        if (fixed_batches) {
            B = P->hbm_batch[gi];
        } else {
            if (budget < per_item) {
                msg = "one " + std::to_string(k) + "-qubit item needs " + std::to_string(per_item) +
                      " bytes, more than the memory budget of " + std::to_string(budget);
                return QAOA_ENOMEM;
            }
            B = batch_of(per_item);
        }
        // free memory can be fragmented or held by other allocators: on a failed allocation
        // the batch is halved until one item does not fit either
        for (;;) {
            st = QAOA_OK;
            if (need_phi) st = grow(P->d_phi, P->cap_phi, (static_cast<size_t>(B) * nphi) << kh, msg);
            if (st == QAOA_OK && need_lam) st = grow(P->d_lam, P->cap_lam, static_cast<size_t>(B) << kh, msg);
            if (st == QAOA_OK) st = grow(P->d_gpart, P->cap_gpart, static_cast<size_t>(B) * tiles * stride, msg);
            if (st != QAOA_ENOMEM || B == 1) break;
            for (float2** b : {&P->d_phi, &P->d_lam}) {
                hipFree(*b);
                *b = nullptr;
            }
            P->cap_phi = P->cap_lam = 0;
            B /= 2;
        }
        if (st != QAOA_OK) return st;
        P->hbm_batch[gi] = B;
        P->hbm_ckpt[gi] = ckpt ? 1 : 0;
        if (!fixed_batches && ckpt) {
            P->checkpointed_classes += 1;
            P->checkpointed_k_mask |= 1u << k;
        }
        const std::vector<PassSpec> prog = hbm_program(k, p, grad, ckpt);
        auto slot = [&](int j) { return P->d_phi + ((static_cast<size_t>(std::max(j, 0)) * B) << kh); };
        QCHECK(tm.begin(k, items));
        auto pass_args = [&](const PassSpec& ps, int64_t i0, int64_t nb) {
            PassArgs pa{};
            pa.cones = P->d_hcones + grp.first;
            pa.e_a = P->d_ea;
            pa.e_b = P->d_eb;
            pa.e_w = P->d_ew;
            pa.e_wd = P->d_ewd;
            pa.tt = P->d_tt;
            pa.phi_in = slot(ps.ck_in);
            pa.phi = ps.kind >= RV_GEN_MIX ? slot(ps.ck_in) : slot(ps.ck_out);
            pa.store_phi = ps.store_phi;
            pa.lam = P->d_lam;
            pa.gpart = P->d_gpart;
            pa.item0 = i0;
            pa.n_batch = static_cast<int32_t>(nb);
            pa.k = k;
            pa.kh = kh;
            pa.group = ps.group;
            pa.la = ps.la;
            pa.lb = ps.lb;
            pa.m0a = ps.m0a;
            pa.m0b = ps.m0b;
            pa.rowcap = grp.rowcap;
            pa.fix_layer = ps.fix_layer;
            pa.fix_pow = ps.fix_pow;
            pa.tpw = tpw;
            pa.ea = ea;
            return pa;
        };
        if (tune_tpw) {
            // tiles per workgroup: the class's first pass on its first batch (a generating
            // pass: it reads no state, and the partial sums it adds are cleared below)
            std::vector<int> cand;
            const int64_t units = tiles / 2;   // tile pairs of group 0 (the fewest units)
            for (int c = 1; c <= 8; c *= 2)
                if (c <= units && units % c == 0) cand.push_back(c);
            const int64_t nb = std::min<int64_t>(B, items);
            QCHECK(tune_pick(tkey, cand, nb, stream, [&](int c) {
                PassArgs pa = pass_args(prog[0], 0, nb);
                pa.tpw = c;
                return launch_pass(prog[0].kind, pa, stream);
            }, tpw));
        }
        for (int64_t i0 = 0; i0 < items; i0 += B) {
            const int64_t nb = std::min<int64_t>(B, items - i0);
            QCHECK(launch_fill_zero(P->d_gpart, nb * tiles * stride, stream));
            for (const PassSpec& ps : prog) {
                const PassArgs pa = pass_args(ps, i0, nb);
                QCHECK(launch_pass(ps.kind, pa, stream));
                if (!fixed_batches) P->pass_launches[ps.kind] += 1;
            }
            QCHECK(launch_tile_reduce(P->d_hcones + grp.first, P->d_gpart, i0, nb, tiles, stride, nvals, ea, stream));
        }
        QCHECK(tm.end());
    }
    QCHECK(tm.begin(-2, n_points));
    if (grad && term_grad) {
        // the caller reads the per-term gradient: gamma derivatives in radians (the combination
        // then scales by the unit once more, so it gets unit weights)
        bool unit = true;
        for (double d : hp.inst_delta) unit = unit && d == 1.0;
        if (!unit) {
            QCHECK(launch_scale_gamma_terms(g, n_points, p, M, P->d_inst_orbit, hp.n_inst, P->d_inst_delta, stream));
        }
        QCHECK(launch_combine(P->d_W, zz, g, M, p, P->d_inst_orbit, unit ? P->d_inst_delta : P->d_ones, hp.n_inst,
                              n_points, n_points, 0, energy, dgamma, dbeta, stream));
    } else {
        QCHECK(launch_combine(P->d_W, zz, g, M, p, P->d_inst_orbit, P->d_inst_delta, hp.n_inst, n_points, n_points,
                              0, energy, dgamma, dbeta, stream));
    }
    QCHECK(tm.end());
    return QAOA_OK;
}

void drop_graph(qaoa_plan_s* P) {
    if (P->gexec) hipGraphExecDestroy(P->gexec);
    P->gexec = nullptr;
    P->gkey = qaoa_plan_s::GraphKey{};
}

}  // namespace

qaoa_status run_energy(qaoa_plan_s* P, int64_t n_points, const double* gamma, const double* beta, double* energy,
                       double* term_zz, double* dgamma, double* dbeta, double* term_grad, hipStream_t stream,
                       std::string& msg) {
    if (!P->opt.graph)
        return enqueue(P, n_points, gamma, beta, energy, term_zz, dgamma, dbeta, term_grad, stream, false, msg);
    qaoa_plan_s::GraphKey key;
    key.n_points = n_points;
    key.grad = dgamma != nullptr;
    const void* ptrs[7] = {gamma, beta, energy, term_zz, dgamma, dbeta, term_grad};
    for (int i = 0; i < 7; ++i) key.ptr[i] = ptrs[i];
    if (P->gexec && key == P->gkey) {
        QCHECK(hipGraphLaunch(P->gexec, stream));
        ++P->graph_replays;
        return QAOA_OK;
    }
    // a new key: run eagerly (allocating what the call needs), then capture the same launch
    // sequence on the plan's own stream; the graph is replayed from the next call on
    drop_graph(P);
    qaoa_status st = enqueue(P, n_points, gamma, beta, energy, term_zz, dgamma, dbeta, term_grad, stream, false, msg);
    if (st != QAOA_OK) return st;
    if (!P->cap_stream) QCHECK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    QCHECK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    st = enqueue(P, n_points, gamma, beta, energy, term_zz, dgamma, dbeta, term_grad, P->cap_stream, true, msg);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(P->cap_stream, &graph);
    if (st == QAOA_OK && ec != hipSuccess) {
        msg = std::string("hipStreamEndCapture: ") + hipGetErrorString(ec);
        st = QAOA_EHIP;
    }
    if (st == QAOA_OK) {
        const hipError_t ei = hipGraphInstantiate(&P->gexec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            msg = std::string("hipGraphInstantiate: ") + hipGetErrorString(ei);
            P->gexec = nullptr;
            st = QAOA_EHIP;
        }
    }
    if (graph) hipGraphDestroy(graph);
    if (st == QAOA_OK) P->gkey = key;
    return st;
}

std::string tuning_report() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::string out;
    char line[256];
    for (const auto& kv : g_tune) {
        const TuneKey& key = kv.first;
        const TuneRec& r = kv.second;
        std::snprintf(line, sizeof(line), "%s %s k=%d p=%d grad=%d realw=%d items=%lld choice=%d ms:",
                      key.arch.c_str(), key.what == 0 ? "workgroup-variant" : "passes-tiles-per-workgroup", key.k,
                      key.p, key.grad, key.realw, static_cast<long long>(r.items), r.choice);
        out += line;
        for (const auto& cm : r.ms) {
            std::snprintf(line, sizeof(line), " %d=%.4f", cm.first, cm.second);
            out += line;
        }
        out += "\n";
    }
    return out;
}

void release_device(qaoa_plan_s* P) {
    drop_graph(P);
    if (P->cap_stream) {
        hipStreamDestroy(P->cap_stream);
        P->cap_stream = nullptr;
    }
    for (auto& t : P->timed) {
        hipEventDestroy(t.start);
        hipEventDestroy(t.stop);
    }
    P->timed.clear();
    if (!P->dev_ready && !P->d_phase) return;
    hipDeviceSynchronize();
    hipFree(P->d_arena);
    hipFree(P->d_phase);
    hipFree(P->d_mix);
    hipFree(P->d_zz);
    hipFree(P->d_g);
    hipFree(P->d_phi);
    hipFree(P->d_lam);
    hipFree(P->d_gpart);
    P->d_arena = nullptr;
    P->d_cones = nullptr;
    P->d_cut = nullptr;
    P->d_W = nullptr;
    P->d_hcones = nullptr;
    P->d_ea = P->d_eb = P->d_ew = nullptr;
    P->d_ewd = nullptr;
    P->d_tt = nullptr;
    P->d_inst_orbit = nullptr;
    P->d_inst_delta = nullptr;
    P->d_ones = nullptr;
    P->d_phi = P->d_lam = nullptr;
    P->d_gpart = nullptr;
    P->cap_phi = P->cap_lam = P->cap_gpart = 0;
    P->d_phase = nullptr;
    P->d_mix = nullptr;
    P->d_zz = nullptr;
    P->d_g = nullptr;
    P->cap_phase = P->cap_mix = P->cap_zz = P->cap_g = 0;
    P->dev_ready = false;
}

}  // namespace qaoa

// C ABI of libqaoa.so and the per-plan device runtime behind it.
#include "qaoa.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device.hpp"
#include "plan.hpp"
#include "runtime.hpp"

namespace {
thread_local std::string g_last_error;

qaoa_status set_err(qaoa_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}
}  // namespace

namespace qaoa {
qaoa_status set_last_error(qaoa_status st, const std::string& msg) { return set_err(st, msg); }
void clear_last_error() { g_last_error.clear(); }
}  // namespace qaoa

extern "C" {

void qaoa_plan_opts_default(qaoa_plan_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->reduce = 1;
    o->max_cone_qubits = 30;
    o->k_lds_max = 14;
}

const char* qaoa_last_error(void) { return g_last_error.c_str(); }

qaoa_status qaoa_find_generators(const qaoa_problem* pr, int32_t max_generators, double time_limit_s,
                                 int32_t* generators, int32_t* n_found, int32_t* complete) {
    if (!pr || !n_found || !complete || (max_generators > 0 && !generators))
        return set_err(QAOA_EINVAL, "NULL argument");
    if (max_generators < 0 || !(time_limit_s > 0.0)) return set_err(QAOA_EINVAL, "bad limits");
    try {
        std::vector<std::vector<int32_t>> gens;
        bool done = false;
        std::string msg;
        const int64_t leaf_budget = int64_t{1} << 20;
        if (qaoa::find_generators(pr->n_nodes, pr->n_edges, pr->edge_u, pr->edge_v, pr->edge_w, max_generators,
                                  time_limit_s, leaf_budget, gens, done, msg) != 0)
            return set_err(QAOA_EINVAL, msg);
        for (size_t g = 0; g < gens.size(); ++g)
            std::memcpy(generators + g * static_cast<size_t>(pr->n_nodes), gens[g].data(),
                        sizeof(int32_t) * static_cast<size_t>(pr->n_nodes));
        *n_found = static_cast<int32_t>(gens.size());
        *complete = done ? 1 : 0;
        return QAOA_OK;
    } catch (const std::bad_alloc&) {
        return set_err(QAOA_ENOMEM, "host allocation failed");
    }
}

namespace {
qaoa_status plan_options(const qaoa_plan_opts* opts, qaoa::PlanOptions& o) {
    if (opts) {
        o.mem_budget_bytes = opts->mem_budget_bytes;
        o.reduce = opts->reduce;
        o.max_cone_qubits = opts->max_cone_qubits ? opts->max_cone_qubits : 30;
        o.k_lds_max = opts->k_lds_max ? opts->k_lds_max : 14;
        o.checkpoint_mode = opts->checkpoint_mode;
        o.one_cone_at_a_time = opts->one_cone_at_a_time;
        o.profile = opts->profile;
        o.graph = opts->graph;
        o.tune = opts->tune;
        if (o.tune < 0 || o.tune > 5) return set_err(QAOA_EINVAL, "tune must be 0, 1 or 2-5");
        if (o.mem_budget_bytes < 0) return set_err(QAOA_EINVAL, "mem_budget_bytes must be >= 0");
        if (o.reduce != 0 && o.reduce != 1) return set_err(QAOA_EINVAL, "reduce must be 0 or 1");
        if (o.graph != 0 && o.graph != 1) return set_err(QAOA_EINVAL, "graph must be 0 or 1");
        if (o.graph && (o.profile || o.one_cone_at_a_time))
            return set_err(QAOA_EINVAL, "graph replay cannot be combined with profile or one_cone_at_a_time");
        if (o.checkpoint_mode < 0 || o.checkpoint_mode > 2)
            return set_err(QAOA_EINVAL, "checkpoint_mode must be 0 (uncompute), 1 (store) or 2 (auto)");
    }
    return QAOA_OK;
}

qaoa_status make_plan(const qaoa_problem* pr, int32_t n_inst, const qaoa_plan_opts* opts, qaoa_plan_t* out) {
    if (!pr || !out) return set_err(QAOA_EINVAL, "problems or out is NULL");
    *out = nullptr;
    if (n_inst < 1) return set_err(QAOA_EINVAL, "n_instances must be >= 1");
    qaoa::PlanOptions o;
    const qaoa_status so = plan_options(opts, o);
    if (so != QAOA_OK) return so;
    int32_t j = 0;
    try {
        auto* plan = new qaoa_plan_s();
        try {
            if (n_inst == 1) {
                qaoa::build_host_plan(pr->n_nodes, pr->n_edges, pr->edge_u, pr->edge_v, pr->edge_w, pr->n_generators,
                                      pr->generators, pr->p, o, plan->hp);
            } else {
                std::vector<qaoa::HostPlan> parts(static_cast<size_t>(n_inst));
                for (j = 0; j < n_inst; ++j) {
                    const qaoa_problem& q = pr[j];
                    qaoa::build_host_plan(q.n_nodes, q.n_edges, q.edge_u, q.edge_v, q.edge_w, q.n_generators,
                                          q.generators, q.p, o, parts[j]);
                }
                j = -1;
                qaoa::merge_host_plans(parts, plan->hp);
            }
        } catch (...) {
            delete plan;
            throw;
        }
        plan->opt = o;
        *out = plan;
        g_last_error.clear();
        return QAOA_OK;
    } catch (const qaoa::PlanError& e) {
        return set_err(e.status, (n_inst > 1 && j >= 0 ? "instance " + std::to_string(j) + ": " : std::string()) + e.msg);
    } catch (const std::bad_alloc&) {
        return set_err(QAOA_ENOMEM, "host allocation failed while planning");
    }
}
}  // namespace

qaoa_status qaoa_plan_lightcones(const qaoa_problem* pr, const qaoa_plan_opts* opts, qaoa_plan_t* out) {
    return make_plan(pr, 1, opts, out);
}

qaoa_status qaoa_plan_batch(const qaoa_problem* problems, int32_t n_instances, const qaoa_plan_opts* opts,
                            qaoa_plan_t* out) {
    return make_plan(problems, n_instances, opts, out);
}

qaoa_status qaoa_plan_query(qaoa_plan_t plan, qaoa_plan_info* out) {
    if (!plan || !out) return set_err(QAOA_EINVAL, "plan or out is NULL");
    const auto& hp = plan->hp;
    std::memset(out, 0, sizeof(*out));
    out->n_nodes = hp.n;
    out->p = hp.p;
    out->n_edges = hp.m;
    out->n_orbits = static_cast<int64_t>(hp.rep.size());
    out->min_k = hp.cones.empty() ? 0 : 31;
    for (const auto& c : hp.cones) {
        out->k_hist[c.k] += 1;
        out->min_k = std::min(out->min_k, c.k);
        out->max_k = std::max(out->max_k, c.k);
        if (c.k > plan->opt.k_lds_max) out->n_hbm_cones += 1;
    }
    out->total_weight = hp.total_weight;
    out->cut_min = hp.cut_min;
    out->cut_max = hp.cut_max;
    out->device_bytes = static_cast<int64_t>(plan->resident_bytes);
    out->graph_replays = plan->graph_replays;
    out->weight_unit = plan->hp.realw ? 0.0 : plan->hp.delta;
    out->real_weights = plan->hp.realw ? 1 : 0;
    for (int i = 0; i < 10 && i < qaoa::N_PASS_KINDS; ++i) out->pass_launches[i] = plan->pass_launches[i];
    out->checkpointed_classes = plan->checkpointed_classes;
    out->checkpointed_k_mask = plan->checkpointed_k_mask;
    out->n_instances = hp.n_inst;
    return QAOA_OK;
}

qaoa_status qaoa_plan_orbits(qaoa_plan_t plan, int32_t* edge_orbit, int64_t* orbit_rep, int64_t* orbit_size) {
    if (!plan) return set_err(QAOA_EINVAL, "plan is NULL");
    const auto& hp = plan->hp;
    if (edge_orbit) std::copy(hp.edge_orbit.begin(), hp.edge_orbit.end(), edge_orbit);
    if (orbit_rep) std::copy(hp.rep.begin(), hp.rep.end(), orbit_rep);
    if (orbit_size) std::copy(hp.size.begin(), hp.size.end(), orbit_size);
    return QAOA_OK;
}

qaoa_status qaoa_plan_cone(qaoa_plan_t plan, int64_t orbit, int32_t* k_out, int32_t* nodes, int32_t capacity,
                           int32_t* n_cone_edges) {
    if (!plan) return set_err(QAOA_EINVAL, "plan is NULL");
    if (orbit < 0 || orbit >= static_cast<int64_t>(plan->hp.cones.size())) return set_err(QAOA_EINVAL, "orbit out of range");
    const auto& c = plan->hp.cones[orbit];
    if (k_out) *k_out = c.k;
    if (nodes && capacity > 0) std::copy_n(c.nodes.begin(), std::min<int32_t>(capacity, c.k), nodes);
    if (n_cone_edges) *n_cone_edges = static_cast<int32_t>(c.ea.size());
    return QAOA_OK;
}

qaoa_status qaoa_energy(qaoa_plan_t plan, int64_t n_points, const double* gamma, const double* beta,
                        double* energy, double* term_zz, qaoa_stream_t stream) {
    if (!plan) return set_err(QAOA_EINVAL, "plan is NULL");
    if (n_points < 1 || n_points > (int64_t{1} << 30)) return set_err(QAOA_EINVAL, "n_points must be in [1, 2^30]");
    if (!gamma || !beta || !energy) return set_err(QAOA_EINVAL, "gamma, beta and energy must be device pointers");
    std::string msg;
    const qaoa_status st = qaoa::run_energy(plan, n_points, gamma, beta, energy, term_zz, nullptr, nullptr, nullptr,
                                            reinterpret_cast<hipStream_t>(stream), msg);
    if (st != QAOA_OK) return set_err(st, msg);
    g_last_error.clear();
    return QAOA_OK;
}

qaoa_status qaoa_energy_grad(qaoa_plan_t plan, int64_t n_points, const double* gamma, const double* beta,
                             double* energy, double* dgamma, double* dbeta, qaoa_stream_t stream) {
    if (!plan) return set_err(QAOA_EINVAL, "plan is NULL");
    if (n_points < 1 || n_points > (int64_t{1} << 30)) return set_err(QAOA_EINVAL, "n_points must be in [1, 2^30]");
    if (!gamma || !beta || !energy || !dgamma || !dbeta)
        return set_err(QAOA_EINVAL, "gamma, beta, energy, dgamma and dbeta must be device pointers");
    std::string msg;
    const qaoa_status st = qaoa::run_energy(plan, n_points, gamma, beta, energy, nullptr, dgamma, dbeta, nullptr,
                                            reinterpret_cast<hipStream_t>(stream), msg);
    if (st != QAOA_OK) return set_err(st, msg);
    g_last_error.clear();
    return QAOA_OK;
}

qaoa_status qaoa_energy_grad_terms(qaoa_plan_t plan, int64_t n_points, const double* gamma, const double* beta,
                                   double* energy, double* dgamma, double* dbeta, double* term_zz,
                                   double* term_grad, qaoa_stream_t stream) {
    if (!plan) return set_err(QAOA_EINVAL, "plan is NULL");
    if (n_points < 1 || n_points > (int64_t{1} << 30)) return set_err(QAOA_EINVAL, "n_points must be in [1, 2^30]");
    if (!gamma || !beta || !energy || !dgamma || !dbeta)
        return set_err(QAOA_EINVAL, "gamma, beta, energy, dgamma and dbeta must be device pointers");
    std::string msg;
    const qaoa_status st = qaoa::run_energy(plan, n_points, gamma, beta, energy, term_zz, dgamma, dbeta, term_grad,
                                            reinterpret_cast<hipStream_t>(stream), msg);
    if (st != QAOA_OK) return set_err(st, msg);
    g_last_error.clear();
    return QAOA_OK;
}

qaoa_status qaoa_plan_kernel_times(qaoa_plan_t plan, int32_t cap, int32_t* k_out, int64_t* items_out,
                                   double* ms_out, int32_t* n_out) {
    if (!plan) return set_err(QAOA_EINVAL, "plan is NULL");
    std::string msg;
    const qaoa_status st = qaoa::kernel_times(plan, cap, k_out, items_out, ms_out, n_out, msg);
    if (st != QAOA_OK) return set_err(st, msg);
    return QAOA_OK;
}

qaoa_status qaoa_tuning_report(char* buf, int64_t cap, int64_t* len) {
    if (!len || (cap > 0 && !buf)) return set_err(QAOA_EINVAL, "len is NULL (or buf is NULL with cap > 0)");
    const std::string r = qaoa::tuning_report();
    *len = static_cast<int64_t>(r.size());
    if (cap > 0) {
        const size_t n = std::min<size_t>(r.size(), static_cast<size_t>(cap - 1));
        std::memcpy(buf, r.data(), n);
        buf[n] = 0;
    }
    return QAOA_OK;
}

void qaoa_plan_destroy(qaoa_plan_t plan) {
    if (!plan) return;
    qaoa::release_device(plan);
    delete plan;
}

}  // extern "C"

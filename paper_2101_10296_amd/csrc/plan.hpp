// Host planner: graph canonicalisation, generator verification, edge orbits and
// light-cone extraction.  Integer-exact; no device code.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace qaoa {

struct PlanError {
    int32_t status;
    std::string msg;
};

// One light cone: the subgraph induced by the radius-p ball around an edge (Sec. 2.3).
struct Cone {
    int32_t k = 0;                         // qubits
    std::vector<int32_t> nodes;            // graph node of each qubit (u, v, then by (dist, id))
    std::vector<int32_t> ea, eb;           // induced edges as qubit pairs, ea < eb
    std::vector<int32_t> ew;               // integer weight of each induced edge (units of delta)
    std::vector<double> wf;                // real weight of each induced edge
    int32_t cut_min = 0, cut_max = 0;      // range of the cut value C(x) over all x (units of delta)
    double cf_min = 0.0, cf_max = 0.0;     // the same range in real weights
    int32_t inst = 0;                      // instance (graph) of a plan over several graphs
};

struct HostPlan {
    int32_t n = 0, p = 0;
    int64_t m = 0;
    std::vector<int32_t> u, v;             // canonical edges, u < v, input order
    std::vector<double> w;                 // weights (1.0 when unit)
    std::vector<int32_t> wi;               // weights in units of delta (integers)
    double delta = 1.0;                    // weight unit: w = delta * wi exactly
    bool unit = true;
    // real weights: no common unit (or a cone's cut values span more than 255 units): cut
    // values are real numbers, the phase of every amplitude is computed from its own cut
    // value; delta = 1 and wi are unused
    bool realw = false;
    std::vector<int32_t> edge_orbit;       // [m]
    std::vector<int64_t> rep, size;        // [M]
    std::vector<double> W;                 // [M] orbit weight = sum of member weights
    std::vector<Cone> cones;               // [M]
    double total_weight = 0.0;
    int32_t cut_min = 0, cut_max = 0;      // over all cones
    // instances: a plan over several graphs is their disjoint union with each graph's nodes,
    // edges and orbits numbered contiguously; weights of instance j count in its own unit
    int32_t n_inst = 1;
    std::vector<int32_t> inst_node;        // [n_inst + 1] first node of each instance
    std::vector<int64_t> inst_edge;        // [n_inst + 1] first edge
    std::vector<int64_t> inst_orbit;       // [n_inst + 1] first orbit
    std::vector<double> inst_delta;        // [n_inst] weight unit of each instance
};

struct PlanOptions {
    int64_t mem_budget_bytes = 0;
    int32_t reduce = 1;
    int32_t max_cone_qubits = 30;
    int32_t k_lds_max = 14;
    int32_t checkpoint_mode = 0;
    int32_t one_cone_at_a_time = 0;
    int32_t profile = 0;
    int32_t graph = 0;
    int32_t tune = 0;
};

// Throws PlanError on invalid input.
void build_host_plan(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* ew,
                     int32_t n_gen, const int32_t* gens, int32_t p, const PlanOptions& opt,
                     HostPlan& out);

// One plan over several graphs of the same depth: the planned instances, concatenated
// (node, edge and orbit ids offset by the sizes of the instances before them).
void merge_host_plans(std::vector<HostPlan>& parts, HostPlan& out);

// Automorphism generators of a weighted graph by individualisation and refinement
// (autgen.cpp).  Returns 0, or -1 with msg on bad input.
int32_t find_generators(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* ew, int32_t max_gens,
                        double seconds, int64_t leaf_budget, std::vector<std::vector<int32_t>>& gens, bool& complete,
                        std::string& msg);

}  // namespace qaoa

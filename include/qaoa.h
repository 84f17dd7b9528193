/*
 * qaoa.h - C ABI of libqaoa.so: symmetry-reduced light-cone QAOA MaxCut energy and
 * its gradient on one AMD Instinct MI355X (gfx950).
 *
 * The method (Shaydulin & Wild, "Exploiting Symmetry Reduces the Cost of Training
 * QAOA", arXiv:2101.10296):
 *   - QAOA state |beta,gamma>_p = U_B(beta_p) U_P(gamma_p) ... U_B(beta_1) U_P(gamma_1) |+>^n
 *     with U_P(gamma) = exp(-i gamma H), U_B(beta) = prod_j exp(-i beta X_j)   (Sec. 2.2)
 *   - MaxCut H = 1/2 sum_{(u,v) in E} w_uv (I - Z_u Z_v)                      (Sec. 2.4;
 *     weights J_uv as in Sec. 4, Eq. 6)
 *   - each term <Z_u Z_v> is evaluated on its reverse causal cone, the radius-p ball
 *     around {u, v}                                                             (Sec. 2.3)
 *   - terms related by a graph automorphism have equal expectation (Sec. 3, Theorem 1),
 *     so only one representative per edge orbit is evaluated and weighted by the
 *     orbit's total weight                                   (Sec. 3, reduced-energy display)
 *
 * Conventions
 *   - All functions return a qaoa_status; on failure nothing is written to outputs and
 *     qaoa_last_error() returns a thread-local description.
 *   - The caller owns every buffer passed in.  qaoa_plan_lightcones copies what it needs;
 *     host inputs may be freed as soon as it returns.
 *   - Angle and output pointers of qaoa_energy / qaoa_energy_grad are DEVICE pointers on
 *     the current HIP device.  Work is enqueued on `stream` (NULL = default stream) and
 *     the outputs are valid once that stream has been synchronised.
 *   - One energy call may be in flight per plan (the plan owns its scratch buffers).
 *   - Angle layout: gamma[i * p + l], beta[i * p + l] for point i and layer l (0-based).
 *   - Energy returned: E(gamma, beta) = <H_MaxCut> = sum_m W_m (1 - zz_m) / 2 with
 *     zz_m = <Z_u Z_v> of the representative of orbit m and W_m the sum of the weights
 *     of the orbit's edges.  The phase on |x> is exp(-i gamma C(x)) with C(x) the weighted
 *     cut (the paper's U_P with H = H_MaxCut); a convention exp(-i g' sum w ZZ) maps to
 *     gamma = -2 g' up to a global phase.
 */
#ifndef QAOA_H
#define QAOA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qaoa_status;
enum {
    QAOA_OK = 0,
    QAOA_EINVAL = -1,   /* bad sizes or ids, self-loop, duplicate edge, p outside [1, 1024],
                           n_points outside [1, 2^30], non-finite weights */
    QAOA_ENOTAUT = -2,  /* a generator is not a weight-preserving automorphism */
    QAOA_ECONE = -3,    /* a light cone exceeds max_cone_qubits */
    QAOA_ENOMEM = -4,   /* not even one work item fits the memory budget / device memory */
    QAOA_EHIP = -5      /* HIP runtime error (no device, launch failure, ...) */
};

/* HIP stream handle; the same type as hipStream_t. */
typedef struct ihipStream_t* qaoa_stream_t;

/* Opaque plan, owned by the library until qaoa_plan_destroy. */
typedef struct qaoa_plan_s* qaoa_plan_t;

/* Problem statement (Sec. 2.4 graph, Sec. 4 weights, Sec. 2.2 depth, Sec. 3 symmetry
 * group given by generators).  All pointers are HOST memory. */
typedef struct {
    int32_t n_nodes;              /* |V| >= 1 */
    int64_t n_edges;              /* |E| >= 0; the input order is the edge index */
    const int32_t* edge_u;        /* [n_edges], 0 <= id < n_nodes */
    const int32_t* edge_v;        /* [n_edges] */
    const double* edge_w;         /* [n_edges] finite weights, or NULL = unit weights.  Weights
                                     that are integer multiples of one common unit (integers,
                                     or rationals with denominators up to 2^20 to 1e-13
                                     relative, at most 2^24 units each) with cut values
                                     spanning at most 255 units per cone use integer cut
                                     tables; any other weights (irrational, Gaussian
                                     couplings, wide ranges) use real cut values per
                                     amplitude (qaoa_plan_info.real_weights) */
    int32_t n_generators;         /* >= 0 */
    const int32_t* generators;    /* row-major [n_generators][n_nodes]: image of node i under
                                     generator g; NULL / 0 = trivial group */
    int32_t p;                    /* QAOA depth, 1 <= p <= 1024 */
} qaoa_problem;

/* Planning options.  Pass NULL for the defaults (qaoa_plan_opts_default). */
typedef struct {
    int64_t mem_budget_bytes;     /* device bytes the plan may use for cone states held in
                                     device memory; 0 = 85 % of free device memory at first
                                     use.  Items are batched within it, at most as many per
                                     batch as give 2^17 workgroups per pass */
    int32_t reduce;               /* 1 = one term per edge orbit (default); 0 = every edge is
                                     its own term (the plain, unreduced light-cone sum) */
    int32_t max_cone_qubits;      /* 0 = 30 */
    int32_t k_lds_max;            /* cones with k <= this run entirely inside one workgroup,
                                     larger ones as passes over tiles held in device memory
                                     (0 = default; only 14 is accepted) */
    int32_t checkpoint_mode;      /* adjoint of cones held in device memory (p >= 2):
                                     0 = uncompute: the forward state is recovered by inverse
                                         layers, two live states per item (default);
                                     1 = store: every forward pass but the final one keeps its
                                         output (one state per pass group and layer), and each
                                         reverse pass reads the state it needs instead of
                                         carrying the uncomputed one (c + 1 live states per item,
                                         c = passes per forward sweep - 1; less traffic, no
                                         FP32 drift of the uncomputation);
                                     2 = auto: store where the memory budget holds the extra
                                         states without fewer items per batch, or with a batch
                                         that still gives every pass 2^15 workgroups; else
                                         uncompute */
    int32_t one_cone_at_a_time;   /* 1 = plain GPU path: one launch per (cone, point) */
    int32_t profile;              /* 1 = record HIP events around every kernel group of each
                                     energy call (read with qaoa_plan_kernel_times) */
    int32_t graph;                /* 1 = replay: the first call with a given (n_points, gradient
                                     or not, device pointers) runs eagerly and captures its launch
                                     sequence into a HIP graph; later calls with the same key
                                     replay the graph on the caller's stream (angle values may
                                     change in place between calls).  Not with profile or
                                     one_cone_at_a_time. */
    int32_t tune;                 /* 1 = run-time tuning: the first call that needs a kernel class
                                     times its layout choices on the device (workgroup-resident
                                     cones: register bits per LDS stage and workgroup size;
                                     cones in device memory: tiles per workgroup) and keeps the
                                     fastest for the rest of the process, per (device
                                     architecture, class, k, p, gradient, real weights);
                                     qaoa_tuning_report lists the choices.  0 = fixed defaults;
                                     2, 3, 4, 5 = workgroup layout 0 (default), 1 (one register
                                     bit fewer per stage), 2 (workgroups of >= 256 threads),
                                     3 (14-qubit adjoint: register/lane exchange layouts, one LDS
                                     transpose per layer) wherever it applies, without timing
                                     (tests, experiments) */
} qaoa_plan_opts;

typedef struct {
    int32_t n_nodes;
    int32_t p;
    int64_t n_edges;
    int64_t n_orbits;             /* M: number of evaluated terms */
    int32_t min_k, max_k;         /* smallest / largest cone (qubits) */
    int64_t k_hist[31];           /* number of cones with k qubits, k = 0..30 */
    double total_weight;          /* sum of all edge weights */
    int32_t cut_min, cut_max;     /* range of cut values over all cones, in weight units */
    int64_t n_hbm_cones;          /* cones too large for one workgroup (state kept in HBM) */
    int64_t device_bytes;         /* descriptor and table bytes resident on the device */
    int64_t graph_replays;        /* energy calls served by replaying a captured graph */
    double weight_unit;           /* delta: every weight is an integer multiple of it (1 for
                                     integer weights); cut values are counted in this unit */
    int64_t pass_launches[10];    /* launches of each device-memory pass kind in the last eagerly
                                     run energy call (all batches), indexed by kind:
                                     0 generate + layer-1 mixer, 1 p = 1 single pass, 2 mixer only,
                                     3 mixer + phase + mixer across a layer boundary, 4 final pass,
                                     5 p = 1 forward + adjoint, 6 final pass + adjoint turn,
                                     7 undo of 0, 8 undo of 2, 9 undo of 3 */
    int32_t checkpointed_classes; /* device-memory cone-size classes whose adjoint read stored
                                     forward states in the last eagerly run call */
    int32_t n_instances;          /* graphs planned together (qaoa_plan_batch), else 1 */
    uint32_t checkpointed_k_mask; /* bit k set: the k-qubit class read stored forward states */
    int32_t real_weights;         /* 1: the weights have no common unit (or a cone's cut values
                                     span more than 255 units): the phase of every amplitude
                                     is computed from its own real cut value (FP64 reduction of
                                     the angle, FP32 sine and cosine); weight_unit is 0 */
} qaoa_plan_info;

void qaoa_plan_opts_default(qaoa_plan_opts* opts);

/* Build a plan: canonicalise the edges (u < v), verify every generator (a permutation of
 * the nodes mapping E onto E and keeping each weight bit for bit: an automorphism of the
 * edge-coloured graph, Sec. 2.6 and Sec. 4), form edge orbits under the group they
 * generate (Sec. 3, Theorem 1: terms of one orbit have equal expectation; representative =
 * smallest edge index, orbits numbered by ascending representative), and extract one
 * light cone per orbit (Sec. 2.3, the reverse causal cone of Z_u Z_v after p layers):
 * qubit 0 = u, qubit 1 = v, the rest of the radius-p ball by (distance, node id); every
 * induced edge is a cone edge.
 * Host-only work; device tables are built on the first energy call.
 * Errors: EINVAL, ENOTAUT, ECONE. */
qaoa_status qaoa_plan_lightcones(const qaoa_problem* problem, const qaoa_plan_opts* opts,
                                 qaoa_plan_t* out);

/* One plan over n_instances >= 1 graphs of the same depth p (problems[j].p equal), each
 * validated, reduced by its own generators and cut into light cones exactly as by
 * qaoa_plan_lightcones; the reduced sum of Sec. 3 is taken per instance.  Every cone of
 * every instance then goes through the same launches: the cones of one size form one batch
 * whatever instance they come from (Sec. 2.3: terms are independent).  Nodes, edges and
 * orbits of instance j are numbered after those of instances 0..j-1 (qaoa_plan_orbits,
 * qaoa_plan_cone, term_zz use these global ids; an instance's orbits are contiguous).
 * Evaluation layouts for a plan with N instances (N = 1: as documented below):
 *   gamma, beta [N][n_points][p] (instance j's points are its own),
 *   energy [N][n_points], dgamma, dbeta [N][n_points][p],
 *   term_zz [n_points][n_orbits], term_grad [n_points][2p][n_orbits] (orbit m of instance j
 *   at instance j's point i).
 * weight_unit in qaoa_plan_info is 0 when the instances' units differ.
 * Errors: as qaoa_plan_lightcones, with the failing instance named in qaoa_last_error. */
qaoa_status qaoa_plan_batch(const qaoa_problem* problems, int32_t n_instances,
                            const qaoa_plan_opts* opts, qaoa_plan_t* out);

/* Summary of a plan (host): sizes of the reduced problem of Sec. 3 (number of orbits M,
 * the cone-size histogram of Sec. 2.3) and device bookkeeping.  out is caller-owned.
 * Errors: EINVAL (NULL argument). */
qaoa_status qaoa_plan_query(qaoa_plan_t plan, qaoa_plan_info* out);

/* Orbit assignment of Sec. 3 (the classes S~_m of equivalent terms and their chosen
 * representatives) into caller-owned host buffers: edge_orbit[n_edges] (orbit of each edge,
 * input order), orbit_rep[n_orbits] (representative edge index), orbit_size[n_orbits]
 * (edges in the orbit).  Any pointer may be NULL.  Errors: EINVAL (NULL plan). */
qaoa_status qaoa_plan_orbits(qaoa_plan_t plan, int32_t* edge_orbit, int64_t* orbit_rep,
                             int64_t* orbit_size);

/* Cone of orbit m (host buffers): *k_out = qubits; nodes[i] = graph node of qubit i
 * (capacity entries are written at most); *n_cone_edges = induced edges.
 * EINVAL if m is out of range. */
qaoa_status qaoa_plan_cone(qaoa_plan_t plan, int64_t orbit, int32_t* k_out, int32_t* nodes,
                           int32_t capacity, int32_t* n_cone_edges);

/* Energy at n_points angle points (Sec. 2.2 ansatz, Sec. 3 reduced sum).
 * gamma, beta: device [n_points * p]; energy: device [n_points];
 * term_zz: device [n_points * n_orbits] (point-major: term_zz[i * n_orbits + m]) or NULL.
 * Errors: EINVAL, ENOMEM, EHIP. */
qaoa_status qaoa_energy(qaoa_plan_t plan, int64_t n_points, const double* gamma,
                        const double* beta, double* energy, double* term_zz,
                        qaoa_stream_t stream);

/* Energy (as qaoa_energy) and its gradient dE/dgamma_l, dE/dbeta_l (device [n_points * p]
 * each, same layout as the angles).  The paper evaluates energies only; training the
 * angles (Sec. 2.2: the angles are optimised classically) needs the gradient, computed
 * here term by term on the same light cones by an adjoint sweep: lambda = Z_u Z_v psi is
 * carried back through the inverse layers, and d<Z_u Z_v>/dbeta_l = 2 Im <lambda|sum_j X_j|psi>,
 * d<Z_u Z_v>/dgamma_l = 2 Im <lambda|H|psi> at layer l.  The forward state is recovered by
 * applying inverse layers (checkpoint_mode 0) or read back from states stored during the
 * forward sweep (see qaoa_plan_opts.checkpoint_mode).
 * Errors: EINVAL, ENOMEM, EHIP. */
qaoa_status qaoa_energy_grad(qaoa_plan_t plan, int64_t n_points, const double* gamma,
                             const double* beta, double* energy, double* dgamma,
                             double* dbeta, qaoa_stream_t stream);

/* qaoa_energy_grad that also returns the per-orbit terms: term_zz as in qaoa_energy, and
 * term_grad: device [n_points * 2p * n_orbits] (point-major, then parameter, then orbit:
 * term_grad[(i * 2p + j) * n_orbits + m] = d zz_m / d gamma_(j+1) for j < p and
 * d zz_m / d beta_(j-p+1) for j >= p, in radians; the energy gradient is
 * -1/2 sum_m W_m term_grad[..][m], Sec. 3 reduced sum).  Either pointer may be NULL.
 * Errors: EINVAL, ENOMEM, EHIP. */
qaoa_status qaoa_energy_grad_terms(qaoa_plan_t plan, int64_t n_points, const double* gamma,
                                   const double* beta, double* energy, double* dgamma,
                                   double* dbeta, double* term_zz, double* term_grad,
                                   qaoa_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid hipMalloc): qaoa_energy_grad with every
 * per-call buffer (angle tables, per-term values) in a scratch array of
 * QAOA_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on until the process
 * ends.  It calls no hipMalloc or hipFree.  Same arguments and results as qaoa_energy_grad;
 * the points are processed in chunks that fit the array.
 *   - The plan must already be resident on the current device (its first qaoa_energy or
 *     qaoa_energy_grad call there uploads its tables) -> else QAOA_EINVAL.
 *   - Every cone must fit one workgroup (no cone above k_lds_max qubits: larger cones keep
 *     states of 2^(k-1) * 8 bytes in device memory) -> else QAOA_EINVAL.
 *   - One point must fit the array: p * (cut range + 1) * 8 + (2p + 1) * n_orbits * 8 bytes
 *     (plus alignment) <= QAOA_NOALLOC_SCRATCH_BYTES -> else QAOA_EINVAL.
 *   - All calls on one GPU share its array: calls that overlap on one GPU (other streams or
 *     threads) race; calls on one stream are ordered by it.
 * Errors: EINVAL, EHIP. */
#define QAOA_NOALLOC_SCRATCH_BYTES (32u << 20)
qaoa_status qaoa_energy_grad_noalloc(qaoa_plan_t plan, int64_t n_points, const double* gamma,
                                     const double* beta, double* energy, double* dgamma,
                                     double* dbeta, qaoa_stream_t stream);

/* Diagnostics for plans built with opts.profile = 1: per kernel group of the last energy
 * call (one group per cone size k, plus the table and combine kernels, reported with
 * k = -1 and k = -2), the cone size, the number of (cone, point) items and the elapsed
 * milliseconds between HIP events recorded on the call's stream around the group.
 * Blocks until those events have completed.  *n_out = number of groups (at most cap
 * are written).  EINVAL if the plan was not built with profiling or has not run. */
qaoa_status qaoa_plan_kernel_times(qaoa_plan_t plan, int32_t cap, int32_t* k_out, int64_t* items_out,
                                   double* ms_out, int32_t* n_out);

/* Automorphism generators of the problem's graph (edge weights act as edge colours), for
 * graphs whose symmetry group is not known by construction; the paper obtains its group
 * from an automorphism solver (Sec. 2.6, Sec. 5).  Colour refinement and
 * individualisation; every permutation written is a verified weight-preserving automorphism
 * and can be passed as problem->generators.
 *   pr->n_nodes, n_edges, edge_u, edge_v, edge_w are read; generators and p are ignored.
 *   max_generators   capacity of `generators`
 *   time_limit_s     wall-clock limit of the search (> 0)
 *   generators       HOST [max_generators][n_nodes], caller-owned: image of node i under g
 *   n_found          number of generators written
 *   complete         1 if the search finished (the generators generate the automorphism
 *                    group), 0 if a limit ended it (they generate a subgroup)
 * Errors: QAOA_EINVAL for a bad graph (ids, self-loops, duplicate edges) or limits. */
qaoa_status qaoa_find_generators(const qaoa_problem* pr, int32_t max_generators, double time_limit_s,
                                 int32_t* generators, int32_t* n_found, int32_t* complete);

/* The run-time tuner's choices so far in this process (plans built with opts.tune = 1), one
 * line per kernel class: device architecture, class, k, p, gradient, real weights, the
 * chosen layout and the milliseconds measured for every candidate.  Writes at most cap - 1
 * characters and a terminating zero into buf (caller-owned host memory, may be NULL when
 * cap is 0); *len = the length of the whole report.  The tuner serves the batching and
 * scheduling of the light-cone evaluations (Sec. 2.3 terms are independent work items).
 * Errors: EINVAL (NULL len). */
qaoa_status qaoa_tuning_report(char* buf, int64_t cap, int64_t* len);

/* Release the plan and everything it owns on the device (synchronises the device). */
void qaoa_plan_destroy(qaoa_plan_t plan);

/* Text of the last failure on this thread ("" if none). */
const char* qaoa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QAOA_H */

// Energy and gradient without any device allocation: the per-call scratch (angle tables and
// the per-term values) lives in one file-scope device array, sized once for the library.
//
// The array is a module global: every GPU the library runs on holds its own copy (at its
// own address) until the process ends.  In host code its name is only a host-side stand-in,
// so the device address is looked up once per device with hipGetSymbolAddress and every
// kernel argument uses that address.  All calls on one GPU share that GPU's copy: calls
// that overlap on one GPU (different streams or threads) race and must be serialised by the
// caller; calls on one stream are ordered by the stream.  Nothing in the array has to start
// at zero: every slot a kernel reads was written earlier in the same call.
#include <mutex>

#include "runtime.hpp"

namespace qaoa {
namespace {

constexpr size_t kScratchBytes = QAOA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on the first call per device).
qaoa_status scratch_of(int dev, void** out, std::string& msg) {
    if (dev < 0 || dev >= kMaxDevices) {
        msg = "device index " + std::to_string(dev) + " beyond the " + std::to_string(kMaxDevices) + " supported";
        return QAOA_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return QAOA_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return QAOA_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t{255}; }

}  // namespace

qaoa_status run_energy_grad_noalloc(qaoa_plan_s* P, int64_t n_points, const double* gamma, const double* beta,
                                    double* energy, double* dgamma, double* dbeta, hipStream_t stream,
                                    std::string& msg) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        msg = std::string("no HIP device: ") + hipGetErrorString(e);
        return QAOA_EHIP;
    }
    if (!P->dev_ready || P->device != dev) {
        msg = "the plan is not resident on the current device: its tables are uploaded by a first "
              "qaoa_energy or qaoa_energy_grad call on this device";
        return QAOA_EINVAL;
    }
    if (!P->hbm_groups.empty()) {
        msg = "the plan has light cones held in device memory (more than " + std::to_string(P->opt.k_lds_max) +
              " qubits); their states need allocations";
        return QAOA_EINVAL;
    }
    void* base = nullptr;
    qaoa_status st = scratch_of(dev, &base, msg);
    if (st != QAOA_OK) return st;

    const HostPlan& hp = P->hp;
    const int32_t p = hp.p;
    const int32_t M = static_cast<int32_t>(hp.cones.size());
    const int32_t R = hp.cut_max - hp.cut_min + 1;
    const int32_t ni = hp.n_inst;
    // bytes per angle point (of every instance): phase rows, mixer factors, zz and the
    // per-term gradient
    const size_t b_phase = static_cast<size_t>(ni) * p * R * sizeof(float2);
    const size_t b_mix = static_cast<size_t>(ni) * p * sizeof(float2);
    const size_t b_zz = static_cast<size_t>(M) * sizeof(double);
    const size_t b_g = static_cast<size_t>(2) * p * M * sizeof(double);
    const size_t per_point = b_phase + b_mix + b_zz + b_g;
    const size_t usable = kScratchBytes - 4 * 256;   // room for aligning four regions
    const int64_t chunk = std::min<int64_t>(n_points, static_cast<int64_t>(usable / per_point));
    if (chunk < 1) {
        msg = "one angle point needs " + std::to_string(per_point) + " bytes of scratch (p = " + std::to_string(p) +
              ", " + std::to_string(M) + " orbits, " + std::to_string(ni) + " instance(s), cut range " +
              std::to_string(R) + "); the buffer holds " + std::to_string(kScratchBytes);
        return QAOA_EINVAL;
    }
    char* s = static_cast<char*>(base);
    float2* phase = reinterpret_cast<float2*>(s);
    float2* mix = reinterpret_cast<float2*>(s + align256(chunk * b_phase));
    double* zz = reinterpret_cast<double*>(reinterpret_cast<char*>(mix) + align256(chunk * b_mix));
    double* g = reinterpret_cast<double*>(reinterpret_cast<char*>(zz) + align256(chunk * b_zz));

#define NCHECK(expr)                                                   \
    do {                                                               \
        const hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) {                                        \
            msg = std::string(#expr) + ": " + hipGetErrorString(e_);   \
            return QAOA_EHIP;                                          \
        }                                                              \
    } while (0)
    for (int64_t i0 = 0; i0 < n_points; i0 += chunk) {
        const int64_t pc = std::min<int64_t>(chunk, n_points - i0);
        // tables [instance][point of the chunk][layer]: one launch per instance (its angles
        // are rows i0 .. i0 + pc - 1 of its [n_points][p] block)
        for (int32_t j = 0; j < ni; ++j) {
            const size_t src = (static_cast<size_t>(j) * n_points + i0) * p;
            const size_t dst = static_cast<size_t>(j) * pc * p;
            NCHECK(launch_tables(gamma + src, beta + src, pc * p, R, hp.cut_min, P->d_inst_delta + j, pc * p,
                                 phase + dst * R, mix + dst, stream));
        }
        // real weights read the angles directly: point i of the chunk is row i0 + i of its
        // instance's block of n_points
        const EvalArgs ea{static_cast<int32_t>(pc), p, M, R, phase, mix, gamma + static_cast<size_t>(i0) * p,
                          static_cast<int32_t>(n_points), hp.realw ? 1 : 0, zz, g};
        for (const auto& grp : P->lds_groups)
            NCHECK(launch_fused(grp.K, true, 0, P->d_cones + grp.first, 0, grp.count * pc, P->d_cut, grp.rowcap,
                                ea, stream));   // default layout: no tuning runs here
        NCHECK(launch_combine(P->d_W, zz, g, M, p, P->d_inst_orbit, P->d_inst_delta, ni, pc, n_points, i0, energy,
                              dgamma, dbeta, stream));
    }
#undef NCHECK
    return QAOA_OK;
}

}  // namespace qaoa

extern "C" qaoa_status qaoa_energy_grad_noalloc(qaoa_plan_t plan, int64_t n_points, const double* gamma,
                                                const double* beta, double* energy, double* dgamma, double* dbeta,
                                                qaoa_stream_t stream) {
    using qaoa::set_last_error;
    if (!plan) return set_last_error(QAOA_EINVAL, "plan is NULL");
    if (n_points < 1 || n_points > (int64_t{1} << 30)) return set_last_error(QAOA_EINVAL, "n_points must be in [1, 2^30]");
    if (!gamma || !beta || !energy || !dgamma || !dbeta)
        return set_last_error(QAOA_EINVAL, "gamma, beta, energy, dgamma and dbeta must be device pointers");
    std::string msg;
    const qaoa_status st = qaoa::run_energy_grad_noalloc(plan, n_points, gamma, beta, energy, dgamma, dbeta,
                                                         reinterpret_cast<hipStream_t>(stream), msg);
    if (st != QAOA_OK) return set_last_error(st, msg);
    qaoa::clear_last_error();
    return QAOA_OK;
}

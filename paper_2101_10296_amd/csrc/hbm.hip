// Launchers of the HBM-resident pass kernels, their per-plan tables and reductions.
#include "hbm_impl.hpp"

namespace qaoa {

// C_tt table of (cone, group): for every tile index q, the weighted cut of the cone edges
// whose two ends lie inside the tile, minus tt_min, as a byte.
__global__ void k_tt_tables(const ConeHbm* __restrict__ cones, const int32_t* __restrict__ ea,
                            const int32_t* __restrict__ eb, const int32_t* __restrict__ ew,
                            uint8_t* __restrict__ tt) {
    const ConeHbm cd = cones[blockIdx.x];
    const int grp = blockIdx.y;
    if (grp >= cd.n_groups) return;
    __shared__ int32_t pos[32];   // tile position of each global bit, -1 if outer
    if (threadIdx.x < 32) pos[threadIdx.x] = -1;
    __syncthreads();
    if (threadIdx.x < HT) {
        int h;
        pos[hgroup_bits(cd.k - 1, grp, threadIdx.x, h)] = threadIdx.x;   // stored qubits
    }
    __syncthreads();
    uint8_t* out = tt + cones[blockIdx.x].tt_off[grp];
    const int32_t tmin = cones[blockIdx.x].tt_min[grp];
    for (uint32_t q = threadIdx.x; q < HN; q += blockDim.x) {
        int32_t c = 0;
        for (int e = 0; e < cd.n_edges; ++e) {
            const int pa = pos[ea[cd.edge_off + e]], pb = pos[eb[cd.edge_off + e]];
            if (pa >= 0 && pb >= 0) c += ew[cd.edge_off + e] * static_cast<int32_t>(((q >> pa) ^ (q >> pb)) & 1u);
        }
        out[q] = static_cast<uint8_t>(c - tmin);
    }
}

// Real weights: the C_tt table of (cone, group) as floats (FP64 sums rounded once).
__global__ void k_tt_tables_real(const ConeHbm* __restrict__ cones, const int32_t* __restrict__ ea,
                                 const int32_t* __restrict__ eb, const double* __restrict__ ew,
                                 float* __restrict__ tt) {
    const ConeHbm cd = cones[blockIdx.x];
    const int grp = blockIdx.y;
    if (grp >= cd.n_groups) return;
    __shared__ int32_t pos[32];
    if (threadIdx.x < 32) pos[threadIdx.x] = -1;
    __syncthreads();
    if (threadIdx.x < HT) {
        int h;
        pos[hgroup_bits(cd.k - 1, grp, threadIdx.x, h)] = threadIdx.x;
    }
    __syncthreads();
    float* out = tt + cones[blockIdx.x].tt_off[grp];
    for (uint32_t q = threadIdx.x; q < HN; q += blockDim.x) {
        double c = 0.0;
        for (int e = 0; e < cd.n_edges; ++e) {
            const int pa = pos[ea[cd.edge_off + e]], pb = pos[eb[cd.edge_off + e]];
            if (pa >= 0 && pb >= 0 && (((q >> pa) ^ (q >> pb)) & 1u)) c += ew[cd.edge_off + e];
        }
        out[q] = static_cast<float>(c);
    }
}

__global__ void k_fill_zero(double* __restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        x[i] = 0.0;
}

// Per item: fixed-order sum over tiles of the partial sums (stride values per tile);
// j = 0 -> zz, j >= 1 -> d zz.  The passes sum over the stored half of the state, so the
// result is doubled.
__global__ void __launch_bounds__(256)
k_tile_reduce(const ConeHbm* __restrict__ cones, const double* __restrict__ gpart, int64_t item0, int64_t tiles,
              int32_t stride, EvalArgs ea) {
    __shared__ double sh[256];
    const int64_t bslot = blockIdx.x;
    const int j = blockIdx.y;
    const int64_t item = item0 + bslot;
    const int64_t cslot = item / ea.P;
    const int point = static_cast<int>(item - cslot * ea.P);
    const int orbit = cones[cslot].orbit;
    const double* src = gpart + static_cast<size_t>(bslot) * tiles * stride + j;
    double acc = 0.0;
    for (int64_t t = threadIdx.x; t < tiles; t += 256) acc += src[t * stride];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (j == 0) ea.zz[static_cast<size_t>(point) * ea.M + orbit] = 2.0 * sh[0];
        else ea.g[(static_cast<size_t>(point) * 2 * ea.p + (j - 1)) * ea.M + orbit] = 2.0 * sh[0];
    }
}

// Each workgroup walks pa.tpw consecutive tiles of one item (set-up once per item, one
// block reduction per workgroup); the caller picks tpw.
template <int KIND, bool G0>
static hipError_t launch_one(const PassArgs& pa, hipStream_t st) {
    constexpr int CF = pass_cf(KIND, G0);
    if (pa.kh != pa.k - 1 || pa.kh < HT + 1) return hipErrorInvalidValue;
    const int64_t tiles = int64_t{1} << (pa.kh - HT);
    const int64_t units = CF >= 2 ? tiles / 2 : tiles;   // tile pairs on group 0
    if (pa.tpw < 1 || units % pa.tpw != 0) return hipErrorInvalidValue;
    const int64_t blocks = units * pa.n_batch / pa.tpw;
    if (pa.ea.realw) {   // real weights: per-amplitude phases, no rows, one LDS buffer
        hipLaunchKernelGGL((k_pass<KIND, G0, false, true>), dim3(static_cast<unsigned>(blocks)), dim3(Hz<CF>::W), 0,
                           st, pa);
        return hipGetLastError();
    }
    const size_t dyn = 3 * static_cast<size_t>(pa.rowcap) * sizeof(float2);   // three phase rows
    if constexpr (CF == 3) {
        // two LDS buffers when they fit beside the phase rows
        static std::atomic<size_t> db_static{0};   // + 1 once queried
        size_t db = db_static.load(std::memory_order_relaxed);
        if (!db) {
            hipFuncAttributes fa{};
            const hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_pass<KIND, G0, true>));
            if (e != hipSuccess) return e;
            db = fa.sharedSizeBytes + 1;
            db_static.store(db, std::memory_order_relaxed);
        }
        if (db - 1 + dyn <= 160 * 1024) {
            hipLaunchKernelGGL((k_pass<KIND, G0, true>), dim3(static_cast<unsigned>(blocks)), dim3(Hz<CF>::W), dyn, st,
                               pa);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_pass<KIND, G0, false>), dim3(static_cast<unsigned>(blocks)), dim3(Hz<CF>::W), dyn, st, pa);
    return hipGetLastError();
}

hipError_t launch_pass(int kind, const PassArgs& pa, hipStream_t st) {
    const bool g0 = pa.group == 0;
    switch (kind) {
        case FWD_GEN_MIX: return g0 ? launch_one<FWD_GEN_MIX, true>(pa, st) : launch_one<FWD_GEN_MIX, false>(pa, st);
        case FWD_GEN_FINAL: return g0 ? launch_one<FWD_GEN_FINAL, true>(pa, st) : hipErrorInvalidValue;
        case FWD_MIX: return g0 ? launch_one<FWD_MIX, true>(pa, st) : launch_one<FWD_MIX, false>(pa, st);
        case FWD_BND_MIX: return g0 ? launch_one<FWD_BND_MIX, true>(pa, st) : launch_one<FWD_BND_MIX, false>(pa, st);
        case FWD_BND_FINAL: return g0 ? launch_one<FWD_BND_FINAL, true>(pa, st) : hipErrorInvalidValue;
        case GR_GEN_FINAL: return g0 ? launch_one<GR_GEN_FINAL, true>(pa, st) : hipErrorInvalidValue;
        case GR_BND_FINAL: return g0 ? launch_one<GR_BND_FINAL, true>(pa, st) : hipErrorInvalidValue;
        case RV_GEN_MIX: return g0 ? launch_one<RV_GEN_MIX, true>(pa, st) : launch_one<RV_GEN_MIX, false>(pa, st);
        case RV_MIX: return g0 ? launch_one<RV_MIX, true>(pa, st) : launch_one<RV_MIX, false>(pa, st);
        case RV_BND_MIX: return g0 ? launch_one<RV_BND_MIX, true>(pa, st) : launch_one<RV_BND_MIX, false>(pa, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tt_tables(const ConeHbm* cones, int64_t n_cones, int max_groups, const int32_t* ea,
                            const int32_t* eb, const int32_t* ew, uint8_t* tt, hipStream_t st) {
    if (n_cones <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tt_tables, dim3(static_cast<unsigned>(n_cones), static_cast<unsigned>(max_groups)),
                       dim3(256), 0, st, cones, ea, eb, ew, tt);
    return hipGetLastError();
}

hipError_t launch_tt_tables_real(const ConeHbm* cones, int64_t n_cones, int max_groups, const int32_t* ea,
                                 const int32_t* eb, const double* ew, float* tt, hipStream_t st) {
    if (n_cones <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tt_tables_real, dim3(static_cast<unsigned>(n_cones), static_cast<unsigned>(max_groups)),
                       dim3(256), 0, st, cones, ea, eb, ew, tt);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* x, int64_t n, hipStream_t st) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_zero, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, x, n);
    return hipGetLastError();
}

hipError_t launch_tile_reduce(const ConeHbm* cones, const double* gpart, int64_t item0, int64_t n_batch,
                              int64_t tiles, int32_t stride, int32_t nvals, const EvalArgs& ea, hipStream_t st) {
    // one block per (item, value); a grid holds fewer than 2^32 work-items
    const int64_t CH = static_cast<int64_t>(UINT32_MAX) / (256 * static_cast<int64_t>(nvals));
    for (int64_t b0 = 0; b0 < n_batch; b0 += CH) {
        const unsigned nx = static_cast<unsigned>(n_batch - b0 < CH ? n_batch - b0 : CH);
        hipLaunchKernelGGL(k_tile_reduce, dim3(nx, static_cast<unsigned>(nvals)), dim3(256), 0, st, cones,
                           gpart + static_cast<size_t>(b0) * tiles * stride, item0 + b0, tiles, stride, ea);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace qaoa

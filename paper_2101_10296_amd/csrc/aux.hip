// Small kernels around the light-cone kernels: per-call angle tables, per-plan cut
// tables, and the orbit-weighted combination of term values into E and dE.
#include "device.hpp"

namespace qaoa {

// phase[(i*p + l)*R + j] = exp(-i gamma_{i,l} delta c), c = cmin + j  (U_P on a basis state
// whose cut is delta c, cut values counted in the weight unit delta of the point's instance;
// Sec. 2.2 / 2.4, weights as in Sec. 4), computed in FP64 and rounded to FP32; rows i*p + l
// run over the instances' points (pl_per_inst rows per instance);
// mix[i*p + l] = (tau, |kappa|^2) of exp(-i beta_{i,l} X) = kappa X^e (1 - i tau X) (Sec. 2.2):
// tau = tan beta, |kappa|^2 = cos^2 beta when |cos beta| >= |sin beta|, otherwise
// tau = -cot beta, |kappa|^2 = sin^2 beta.
__global__ void k_tables(const double* __restrict__ gamma, const double* __restrict__ beta,
                         int64_t n_pl, int32_t R, int32_t cmin, const double* __restrict__ deltas,
                         int64_t pl_per_inst, float2* __restrict__ phase, float2* __restrict__ mix) {
    const int64_t total = n_pl * R;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t pl = t / R;
        const int32_t j = static_cast<int32_t>(t - pl * R);
        const double delta = deltas[pl / pl_per_inst];
        double s, c;
        sincos(gamma[pl] * delta * static_cast<double>(cmin + j), &s, &c);
        phase[t] = make_float2(static_cast<float>(c), static_cast<float>(-s));
        if (j == 0) {
            // exp(-i beta X) = kappa X^e (1 - i tau X): the bounded factorisation
            double sb, cb;
            sincos(beta[pl], &sb, &cb);
            double t, k2;
            if (fabs(cb) >= fabs(sb)) {
                t = sb / cb;
                k2 = cb * cb;
            } else {
                t = -cb / sb;
                k2 = sb * sb;
            }
            mix[pl] = make_float2(static_cast<float>(t), static_cast<float>(k2));
        }
    }
}

// Cut table of cone c: table[x] = C(x) - cut_min for every basis state x of its k qubits,
// C(x) = sum over cone edges (a, b) of w_ab [x_a != x_b]  (MaxCut cost, Sec. 2.4).
__global__ void k_cut_tables(const ConeDev* __restrict__ cones, const int32_t* __restrict__ ea,
                             const int32_t* __restrict__ eb, const int32_t* __restrict__ ew,
                             uint8_t* __restrict__ tables) {
    const ConeDev cd = cones[blockIdx.x];
    const uint32_t N = 1u << cd.k;
    uint8_t* out = tables + cd.cut_off;
    for (uint32_t x = threadIdx.x; x < N; x += blockDim.x) {
        int32_t c = 0;
        for (int32_t e = 0; e < cd.n_edges; ++e) {
            const int32_t a = ea[cd.edge_off + e], b = eb[cd.edge_off + e];
            c += ew[cd.edge_off + e] * static_cast<int32_t>(((x >> a) ^ (x >> b)) & 1u);
        }
        out[x] = static_cast<uint8_t>(c - cd.cut_min);
    }
}

// Real-weight cut table of cone c over the stored half (qubit k-1 = 0 for k >= 3):
// table[x] = C(x) - c0 as a float, C(x) = sum over cone edges of w_ab [x_a != x_b] summed
// in FP64 (MaxCut cost with real couplings, Sec. 2.4 and Sec. 4).
__global__ void k_cut_tables_real(const ConeDev* __restrict__ cones, const int32_t* __restrict__ ea,
                                  const int32_t* __restrict__ eb, const double* __restrict__ ew,
                                  float* __restrict__ tables) {
    const ConeDev cd = cones[blockIdx.x];
    const uint32_t N = 1u << (cd.k >= 3 ? cd.k - 1 : cd.k);
    float* out = tables + cd.cut_off;
    for (uint32_t x = threadIdx.x; x < N; x += blockDim.x) {
        double c = 0.0;
        for (int32_t e = 0; e < cd.n_edges; ++e) {
            const int32_t a = ea[cd.edge_off + e], b = eb[cd.edge_off + e];
            if (((x >> a) ^ (x >> b)) & 1u) c += ew[cd.edge_off + e];
        }
        out[x] = static_cast<float>(c - static_cast<double>(cd.c0));
    }
}

hipError_t launch_cut_tables_real(const ConeDev* cones, int64_t n_cones, const int32_t* ea, const int32_t* eb,
                                  const double* ew, float* tables, hipStream_t st) {
    constexpr int64_t CH = static_cast<int64_t>(UINT32_MAX) / 256;
    for (int64_t c0 = 0; c0 < n_cones; c0 += CH) {
        const unsigned nx = static_cast<unsigned>(n_cones - c0 < CH ? n_cones - c0 : CH);
        hipLaunchKernelGGL(k_cut_tables_real, dim3(nx), dim3(256), 0, st, cones + c0, ea, eb, ew, tables);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Per (instance j, point i) block, over the orbits m of instance j:
// block y == 0: energy = sum_m W_m (1 - zz[i][m]) / 2            (Sec. 3 reduced sum)
// block y == 1 + l: -1/2 sum_m W_m g[i][l][m] -> dgamma (l < p, times the instance's weight
// unit: cut values are counted in it) or dbeta (l >= p).
// Term rows i run over the Pc points of this call's chunk; results go to point i0 + i of an
// output with P_out points per instance.  Blocks b0 + blockIdx.x = j * Pc + i.
// Fixed-order reduction (deterministic): thread t sums m = t, t + 256, ...; then a tree.
__global__ void __launch_bounds__(256)
k_combine(const double* __restrict__ W, const double* __restrict__ zz, const double* __restrict__ g,
          int32_t M, int32_t p, const int64_t* __restrict__ inst_orbit, const double* __restrict__ deltas,
          int64_t Pc, int64_t P_out, int64_t i0, int64_t b0, double* __restrict__ energy,
          double* __restrict__ dgamma, double* __restrict__ dbeta) {
    __shared__ double sh[256];
    const int64_t b = b0 + blockIdx.x;
    const int64_t j = b / Pc;
    const int64_t i = b - j * Pc;
    const int y = blockIdx.y;
    const double* src = (y == 0) ? zz + static_cast<size_t>(i) * M
                                 : g + (static_cast<size_t>(i) * 2 * p + (y - 1)) * M;
    const int64_t m0 = inst_orbit[j], m1 = inst_orbit[j + 1];
    double acc = 0.0;
    for (int64_t m = m0 + threadIdx.x; m < m1; m += 256) {
        acc += (y == 0) ? W[m] * (1.0 - src[m]) * 0.5 : -0.5 * W[m] * src[m];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const size_t o = static_cast<size_t>(j) * P_out + i0 + i;
        if (y == 0) energy[o] = sh[0];
        else if (y - 1 < p) dgamma[o * p + (y - 1)] = deltas[j] * sh[0];
        else dbeta[o * p + (y - 1 - p)] = sh[0];
    }
}

hipError_t launch_tables(const double* gamma, const double* beta, int64_t n_pl, int32_t R, int32_t cmin,
                         const double* deltas, int64_t pl_per_inst, float2* phase, float2* mix, hipStream_t st) {
    const int64_t total = n_pl * R;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_tables, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, gamma, beta, n_pl, R,
                       cmin, deltas, pl_per_inst, phase, mix);
    return hipGetLastError();
}

hipError_t launch_cut_tables(const ConeDev* cones, int64_t n_cones, const int32_t* ea, const int32_t* eb,
                             const int32_t* ew, uint8_t* tables, hipStream_t st) {
    // one block per cone; a grid holds fewer than 2^32 threads
    constexpr int64_t CH = static_cast<int64_t>(UINT32_MAX) / 256;
    for (int64_t c0 = 0; c0 < n_cones; c0 += CH) {
        const unsigned nx = static_cast<unsigned>(n_cones - c0 < CH ? n_cones - c0 : CH);
        hipLaunchKernelGGL(k_cut_tables, dim3(nx), dim3(256), 0, st, cones + c0, ea, eb, ew, tables);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// g[i][l][m] *= delta of m's instance for l < p: per-term gamma derivatives from cut values
// counted in the weight unit to radians (only when the caller asks for the per-term gradient).
__global__ void k_scale_gamma_terms(double* __restrict__ g, int64_t P, int32_t p, int32_t M,
                                    const int64_t* __restrict__ inst_orbit, int32_t n_inst,
                                    const double* __restrict__ deltas) {
    const int64_t total = P * p * static_cast<int64_t>(M);
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = t / (static_cast<int64_t>(p) * M);
        const int64_t r = t - i * p * static_cast<int64_t>(M);
        const int64_t m = r % M;
        int32_t lo = 0, hi = n_inst;   // instance j with inst_orbit[j] <= m < inst_orbit[j + 1]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) / 2;
            if (inst_orbit[mid] <= m) lo = mid; else hi = mid;
        }
        g[(i * 2 * p) * static_cast<int64_t>(M) + r] *= deltas[lo];
    }
}

hipError_t launch_scale_gamma_terms(double* g, int64_t P, int32_t p, int32_t M, const int64_t* inst_orbit,
                                    int32_t n_inst, const double* deltas, hipStream_t st) {
    const int64_t total = P * p * static_cast<int64_t>(M);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return hipSuccess;
    hipLaunchKernelGGL(k_scale_gamma_terms, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g, P, p, M,
                       inst_orbit, n_inst, deltas);
    return hipGetLastError();
}

int64_t combine_chunk(uint32_t ny) { return static_cast<int64_t>(UINT32_MAX) / (256 * static_cast<int64_t>(ny)); }

hipError_t launch_combine(const double* W, const double* zz, const double* g, int32_t M, int32_t p,
                          const int64_t* inst_orbit, const double* deltas, int32_t n_inst, int64_t Pc,
                          int64_t P_out, int64_t i0, double* energy, double* dgamma, double* dbeta, hipStream_t st) {
    const unsigned ny = (g != nullptr) ? static_cast<unsigned>(1 + 2 * p) : 1u;
    // one block per (instance, point, value); a grid holds fewer than 2^32 threads
    const int64_t CH = combine_chunk(ny);
    const int64_t nb = static_cast<int64_t>(n_inst) * Pc;
    for (int64_t b0 = 0; b0 < nb; b0 += CH) {
        const unsigned nx = static_cast<unsigned>(nb - b0 < CH ? nb - b0 : CH);
        hipLaunchKernelGGL(k_combine, dim3(nx, ny), dim3(256), 0, st, W, zz, g, M, p, inst_orbit, deltas, Pc, P_out,
                           i0, b0, energy, dgamma, dbeta);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace qaoa

// HBM-resident light cones (more qubits than one workgroup holds): the state of each
// (cone, angle point) item lives in device memory and every layer is applied by passes
// over tiles of 2^13 amplitudes.
//
// Global-flip halving: every cone state is invariant under flipping all k qubits, so only
// the half with qubit k-1 = 0 is stored, on kh = k - 1 qubits; the mixer of qubit k-1
// pairs stored index y with its complement over the kh stored bits.
//
// A pass works on one pass group of stored qubits.  Group 0 holds qubits 0..12 (so qubits
// 0 and 1, u and v, for the final mixer and <Z0 Z1>); group j >= 1 holds up to nine of the
// remaining qubits, 13 + 9(j-1) .. , and carries global bits 0..3 so that every row of a
// tile is 16 contiguous amplitudes (128 bytes).  Tile bits map to global bits through
// gmap; the bits outside the tile select the tile.  Passes of group 0 also apply the mixer
// of qubit k-1: they take the tiles in complementary pairs (T, ~T) and hold tile ~T in
// complemented coordinates (register r of thread tau stands for local index ~q(tau, r)),
// so each amplitude's partner sits in the same register of the other tile.
//
// Layer order (the forward program, built on the host): layers alternate the order in
// which they visit the groups, so that the last group of layer l is the first group of
// layer l+1 and one pass does "finish layer l on this group, phase l+1, start layer l+1
// on this group".  Layer p-1 ends on group 0, whose pass also applies the last phase,
// the mixer on qubits 0 and 1 and <Z0 Z1>.  The adjoint runs the passes backwards,
// undoing the forward operations on psi (read back from the state buffer, which holds the
// forward input of the pass being undone, or recovered by inverse layers) and lambda.
//
// Inside a tile the amplitudes sit in registers in rotated layouts, exactly as in the
// workgroup-resident kernel (fused_impl.hpp), with LDS transposes between layouts; an
// extra I/O layout puts lanes on the contiguous global bits for coalesced loads/stores.
// The cut value of a basis state x = (outer bits o, tile bits q) is
//   C(x) = C_oo(o) + sum_b W1_b(o) + sum_b q_b (WO_b - 2 W1_b(o)) + C_tt(q),
// where b runs over tile bits, WO_b / W1_b are the weights of b's edges to outer bits
// (all of them / those whose outer end is 1 in o), and C_tt is a per-(cone, group) table.
// Qubit k-1 counts as an outer bit fixed at 0.
#pragma once

#include "fused_impl.hpp"

namespace qaoa {

constexpr int HT = 13;                 // tile bits
constexpr uint32_t HN = 1u << HT;      // amplitudes per tile

// Pass kinds.  FWD_* are forward passes; GR_* fuse the final forward pass with the start
// of the adjoint; RV_* undo a forward pass on (psi, lambda).
enum PassKind : int {
    FWD_GEN_MIX = 0,   // D_1 |+>, mixer of layer 1 on the group, store
    FWD_GEN_FINAL,     // p = 1: D_1 |+>, mixer on qubits 0, 1, <Z0 Z1>
    FWD_MIX,           // load, mixer of layer la, store
    FWD_BND_MIX,       // load, mixer la, phase lb = la + 1, mixer lb, store
    FWD_BND_FINAL,     // load, mixer la = p - 1, phase p, last mixer, <Z0 Z1>
    GR_GEN_FINAL,      // p = 1 forward + adjoint, no state buffers
    GR_BND_FINAL,      // FWD_BND_FINAL + adjoint turn: store lambda at the pass input
    RV_GEN_MIX,        // undo FWD_GEN_MIX (gradients of beta_1 share, gamma_1)
    RV_MIX,            // undo FWD_MIX, store psi and lambda
    RV_BND_MIX,        // undo FWD_BND_MIX, store psi and lambda
    N_PASS_KINDS
};

// One HBM-class light cone.
struct ConeHbm {
    int32_t orbit;
    int32_t k;
    int32_t edge_off;
    int32_t n_edges;
    int32_t cut_min;
    int32_t cut_range;
    int32_t n_groups;
    int32_t cut_shift;   // cut_min - plan.cut_min: offset into a phase table row
    int64_t tt_off[4];   // byte offset of the C_tt table of each group
    int32_t tt_min[4];   // value subtracted before storing C_tt as a byte
    int32_t inst;        // instance of the cone (angle tables per instance)
    float c0;            // real weights: centre of the cone's cut range (subtracted from C)
};

struct PassArgs {
    const ConeHbm* cones;      // cones of this k-class
    const int32_t* e_a;        // flattened cone edges (qubit pairs) and weights
    const int32_t* e_b;
    const int32_t* e_w;
    const double* e_wd;        // real weights of the cone edges (plans with real weights)
    const uint8_t* tt;         // C_tt tables (real weights: floats, tt_off counting floats)
    const float2* phi_in;      // state the pass reads [batch][2^kh] (forward input; for a reverse
                               // pass the state at the output of the forward pass it undoes)
    float2* phi;               // state the pass writes [batch][2^kh] (may equal phi_in)
    float2* lam;               // adjoint buffer [batch][2^kh]
    int32_t store_phi;         // reverse passes: 1 = write the undone psi to phi (uncompute),
                               // 0 = do not (psi of the next reverse pass is a stored checkpoint)
    double* gpart;             // per (item, tile) partial sums [batch][tiles][2p + 1]
    int64_t item0;             // first item of the batch (item = slot * P + point)
    int32_t n_batch;           // items in the batch
    int32_t k;                 // cone qubits (same for every cone of the class)
    int32_t kh;                // stored qubits, k - 1
    int32_t group;             // pass group
    int32_t la, lb;            // layers (1-based) of mixer A / phase + mixer B
    int32_t m0a, m0b;          // qubits of layers la / lb undone by earlier reverse passes
    int32_t rowcap;            // phase row capacity (largest cut range)
    int32_t fix_layer;         // > 0: the loaded psi is rescaled by |kappa_fix_layer|^fix_pow
    int32_t fix_pow;
    int32_t tpw;               // tiles (pair passes: tile pairs) per workgroup, a power of two
    EvalArgs ea;
};

// Register configurations (measured on MI355X over 20-30-qubit cones):
//   CF 0  forward, one tile:        32 amplitudes per thread, 256 threads (mixer-only passes
//                                   of groups >= 1)
//   CF 1  one tile:                 16 per state, 512 threads, <= 128 VGPRs (two per CU):
//                                   adjoint passes, and the forward boundary passes (two
//                                   mixers and a phase), which run faster at this occupancy
//   CF 2  tile pair, two states:    16 per tile, 512 threads, <= 128 VGPRs (two per CU):
//                                   forward passes, and the undo of the first forward pass,
//                                   which holds lambda only (30 dwords spill, still 4 % faster
//                                   than one workgroup per CU)
//   CF 3  adjoint, tile pair:       16 per state and tile, 512 threads, one workgroup per CU
//         (four states in registers; fewer amplitudes per thread spill at 1024 threads)
#ifndef QAOA_HBM_CF3_AB
#define QAOA_HBM_CF3_AB 4
#endif
#ifndef QAOA_HBM_CF3_WPE
#define QAOA_HBM_CF3_WPE 2
#endif
template <int CF>
struct Hz {
    static constexpr int AB = CF == 0 ? 5 : (CF == 3 ? QAOA_HBM_CF3_AB : 4);
    static constexpr int A = 1 << AB;
    static constexpr int W = 1 << (HT - AB);        // threads per tile
    static constexpr int WPE = CF == 0 ? 2 : (CF == 3 ? QAOA_HBM_CF3_WPE : 4);   // minimum waves per SIMD
    static constexpr uint32_t NPAD = HN + (HN >> 4) + (HN >> 8) + (AB == 5 ? 2 : 8) * (HN >> 12);   // pad<AB>() buffer
    static constexpr int ROT_IO0 = HT - AB;          // I/O layout of group 0: lanes on tile bits 0..5
    static constexpr int ROT_IOJ = 9 - AB;           // I/O layout of groups >= 1: lanes on tile bits 9..12, 0, 1
};

// Passes that load the next unit's states (tile or tile pair) into registers before working
// on the current one, so that a workgroup's loads overlap its arithmetic: bit KIND for the
// groups >= 1, bit 16 + KIND for group 0.  Only the forward boundary pass of the groups >= 1
// has the registers for it (one state: 80 VGPRs, 108 with the next tile, two workgroups per
// CU kept); measured over 20-30-qubit cones it cut the device-memory time by 4 %.  The
// reverse passes hold two states: with the next unit's they need one workgroup per CU
// (256 VGPRs), and ran 5-12 % slower that way.
#ifndef QAOA_HBM_PF_MASK
#define QAOA_HBM_PF_MASK (1 << FWD_BND_MIX)
#endif
__host__ __device__ constexpr bool pass_pf(int kind, bool g0) {
    return ((QAOA_HBM_PF_MASK >> (kind + (g0 ? 16 : 0))) & 1) != 0;
}

__host__ __device__ constexpr int pass_cf(int kind, bool g0) {
    if (!g0 && kind == FWD_BND_MIX) return 1;
    if (g0 && kind == RV_GEN_MIX) return 2;   // two states (lambda pair; psi_0 regenerated)
    return (kind >= GR_GEN_FINAL ? 1 : 0) + ((g0 && kind != FWD_GEN_FINAL && kind != GR_GEN_FINAL) ? 2 : 0);
}

__device__ constexpr uint32_t rotl13(uint32_t x, int s) {
    s %= HT;
    return s == 0 ? x : (((x << s) | (x >> (HT - s))) & (HN - 1u));
}
template <int CF, int ROT>
__device__ constexpr uint32_t hroff(int r) { return rotl13(static_cast<uint32_t>(r), ROT); }
template <int CF, int ROT>
__device__ __forceinline__ uint32_t htbase(uint32_t tau) { return rotl13(tau << Hz<CF>::AB, ROT); }

template <int CF, int RF, int RT, int A>
__device__ __forceinline__ void hxpose(float2 (&v)[A], float2* xb, uint32_t tau) {
    float2* pf = xb + opaque_u32(pad<Hz<CF>::AB>(htbase<CF, RF>(tau)));
    const float2* pt = xb + opaque_u32(pad<Hz<CF>::AB>(htbase<CF, RT>(tau)));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) pf[pad<Hz<CF>::AB>(hroff<CF, RF>(r))] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) v[r] = pt[pad<Hz<CF>::AB>(hroff<CF, RT>(r))];
}

// psi and lambda through two LDS buffers at once (one barrier pair instead of two).
template <int CF, int RF, int RT, int A>
__device__ __forceinline__ void hxpose_dual(float2 (&f)[A], float2 (&l)[A], float2* xa, float2* xc, uint32_t tau) {
    const uint32_t of = opaque_u32(pad<Hz<CF>::AB>(htbase<CF, RF>(tau)));
    const uint32_t ot = opaque_u32(pad<Hz<CF>::AB>(htbase<CF, RT>(tau)));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        xa[of + pad<Hz<CF>::AB>(hroff<CF, RF>(r))] = f[r];
        xc[of + pad<Hz<CF>::AB>(hroff<CF, RF>(r))] = l[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        f[r] = xa[ot + pad<Hz<CF>::AB>(hroff<CF, RT>(r))];
        l[r] = xc[ot + pad<Hz<CF>::AB>(hroff<CF, RT>(r))];
    }
}

// Mixer on the processed tile bits of layout ROT (tile bit b is processed when bit b of
// pm is set).  Wrapped bits belong to rotation 0.  ALL: every tile bit is processed (group
// 0); otherwise the bits of pm that are clear (a last group with fewer than nine qubits) are
// skipped by a uniform branch.
template <int CF, int ROT, int LB = -1, bool ALL = false, int A>
__device__ __forceinline__ void hmix(float2 (&v)[A], float t, uint32_t pm) {
    constexpr int AB = Hz<CF>::AB;
    if constexpr (LB >= 0) {
        // tile bit LB sits on lane bit 0 of this layout: partner in the neighbouring lane
        if (ALL || ((pm >> LB) & 1u)) {
#pragma unroll
            for (int r = 0; r < A; ++r) {
                const float2 q = lane_x1(v[r]);
                v[r] = make_float2(fmaf(t, q.y, v[r].x), fmaf(-t, q.x, v[r].y));
                if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int i = 0; i < AB; ++i) {
        if (ROT + i >= HT) continue;
        if (!ALL && !((pm >> (ROT + i)) & 1u)) continue;
        int nb = 0;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & (1 << i))) {
                bfly(v[r], v[r | (1 << i)], t);
                if ((++nb & 7) == 0) __builtin_amdgcn_sched_barrier(0);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Undo the mixer on the processed bits of layout ROT for psi and lambda; returns the
// weighted share of Im <lambda| sum_j X_j |psi> (see unmix_stage2).  ALL as in hmix.
template <int CF, int ROT, int LB = -1, bool ALL = false, int A>
__device__ __forceinline__ float hunmix2(float2 (&f)[A], float2 (&l)[A], float t, float k2, float& w, uint32_t pm) {
    constexpr int AB = Hz<CF>::AB;
    float acc = 0.f;
    if constexpr (LB >= 0) {
      if (ALL || ((pm >> LB) & 1u)) {
        // lane bit 0: term on the values before the undo, with the weight before this bit
        const float ti = -t;
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 fq = lane_x1(f[r]);
            const float2 lq = lane_x1(l[r]);
            cacc(a, 1.f, l[r], fq);
            f[r] = make_float2(fmaf(ti, fq.y, f[r].x), fmaf(-ti, fq.x, f[r].y));
            l[r] = make_float2(fmaf(ti, lq.y, l[r].x), fmaf(-ti, lq.x, l[r].y));
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        acc = w * a;
        w = w * k2;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int i = 0; i < AB; ++i) {
        if (ROT + i >= HT) continue;
        if (!ALL && !((pm >> (ROT + i)) & 1u)) continue;
        const float ti = -t;
        float a0 = 0.f, a1 = 0.f;
        int np = 0;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & (1 << i))) {
                const int r2 = r | (1 << i);
                bfly(f[r], f[r2], ti);
                bfly(l[r], l[r2], ti);
                if (np++ & 1) xacc(a1, l[r], l[r2], f[r], f[r2]);
                else xacc(a0, l[r], l[r2], f[r], f[r2]);
                if ((np & 3) == 0) __builtin_amdgcn_sched_barrier(0);
            }
        w *= k2;
        acc = fmaf(w, a0 + a1, acc);
        __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// Processing layouts: rotations 0, AB, 2 AB, ...  Group 0 needs all 13 tile bits,
// groups >= 1 at most 9 (tile bits 0..8).  With NB = S AB + 1 the leftover bit NB-1 is
// lane bit 0 of the last layout and is mixed across lanes there (LB).
template <int CF, bool G0>
struct HStages {
    static constexpr int AB = Hz<CF>::AB;
    static constexpr int NB = G0 ? HT : 9;
    static constexpr bool LQ = NB % AB == 1 && NB / AB >= 2;
    static constexpr int S = LQ ? NB / AB : (NB + AB - 1) / AB;
    static constexpr int LB = LQ ? NB - 1 : -1;
    static constexpr int rot(int s) { return s * AB; }
    static constexpr int IO = G0 ? Hz<CF>::ROT_IO0 : Hz<CF>::ROT_IOJ;
};

// Forward mixer over the group, visiting layouts S-1 .. 0 (DESC) or 0 .. S-1, starting in
// layout FROM_ROT.  Ends in the last visited layout.
template <int CF, bool G0, bool DESC, int FROM_ROT, int A>
__device__ __forceinline__ void hmix_group(float2 (&f)[A], float2* xb, uint32_t tau, float t, uint32_t pm) {
    using H = HStages<CF, G0>;
    static_for<0, H::S>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr int st = DESC ? H::S - 1 - j : j;
        constexpr int prev = (j == 0) ? FROM_ROT : H::rot(DESC ? H::S - j : j - 1);
        if constexpr (prev != H::rot(st)) hxpose<CF, prev, H::rot(st)>(f, xb, tau);
        hmix<CF, H::rot(st), (st == H::S - 1 ? H::LB : -1), G0>(f, t, pm);
    });
}

template <int CF, bool G0, bool DESC, int FROM_ROT, bool DB = false, int A>
__device__ __forceinline__ float hunmix_group(float2 (&f)[A], float2 (&l)[A], float2* xb, uint32_t tau, float t,
                                              float k2, float& w, uint32_t pm, float2* xb2 = nullptr) {
    using H = HStages<CF, G0>;
    float acc = 0.f;
    static_for<0, H::S>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr int st = DESC ? H::S - 1 - j : j;
        constexpr int prev = (j == 0) ? FROM_ROT : H::rot(DESC ? H::S - j : j - 1);
        if constexpr (prev != H::rot(st)) {
            if constexpr (DB) {
                hxpose_dual<CF, prev, H::rot(st)>(f, l, xb, xb2, tau);
            } else {
                hxpose<CF, prev, H::rot(st)>(f, xb, tau);
                hxpose<CF, prev, H::rot(st)>(l, xb, tau);
            }
        }
        acc += hunmix2<CF, H::rot(st), (st == H::S - 1 ? H::LB : -1), G0>(f, l, t, k2, w, pm);
    });
    return acc;
}

// Im <lambda| X_j |psi> for the processed bits j of layout ROT with both states held at one
// point of the layer (no butterfly: X_j commutes with every mixer of the layer, so the
// inner products may be taken anywhere inside it).  ALL as in hmix.
template <int CF, int ROT, int LB = -1, bool ALL = false, int A>
__device__ __forceinline__ float hip_stage(const float2 (&f)[A], const float2 (&l)[A], uint32_t pm) {
    constexpr int AB = Hz<CF>::AB;
    float a0 = 0.f, a1 = 0.f;
    if constexpr (LB >= 0) {
        if (ALL || ((pm >> LB) & 1u)) {
#pragma unroll
            for (int r = 0; r < A; ++r) {
                cacc((r & 1) ? a1 : a0, 1.f, l[r], lane_x1(f[r]));
                if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int i = 0; i < AB; ++i) {
        if (ROT + i >= HT) continue;
        if (!ALL && !((pm >> (ROT + i)) & 1u)) continue;
        int np = 0;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & (1 << i))) {
                const int r2 = r | (1 << i);
                if (np++ & 1) xacc(a1, l[r], l[r2], f[r], f[r2]);
                else xacc(a0, l[r], l[r2], f[r], f[r2]);
                if ((np & 7) == 0) __builtin_amdgcn_sched_barrier(0);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
    return a0 + a1;
}

// The inner products of every processed bit of the group, walking layouts 0 .. S-1 with
// psi and lambda transposed together (one LDS buffer each when DB).  Ends in layout S-1.
template <int CF, bool G0, bool DB = false, int A>
__device__ __forceinline__ float hip_group(float2 (&f)[A], float2 (&l)[A], float2* xb, uint32_t tau, uint32_t pm,
                                           float2* xb2 = nullptr) {
    using H = HStages<CF, G0>;
    float acc = 0.f;
    static_for<0, H::S>([&](auto J) {
        constexpr int st = decltype(J)::value;
        if constexpr (st > 0) {
            if constexpr (DB) {
                hxpose_dual<CF, H::rot(st - 1), H::rot(st)>(f, l, xb, xb2, tau);
            } else {
                hxpose<CF, H::rot(st - 1), H::rot(st)>(f, xb, tau);
                hxpose<CF, H::rot(st - 1), H::rot(st)>(l, xb, tau);
            }
        }
        acc += hip_stage<CF, H::rot(st), (st == H::S - 1 ? H::LB : -1), G0>(f, l, pm);
    });
    return acc;
}

// Undo of the group's mixer on one state (the inverse butterflies only), walking layouts
// S-1 .. 0 from layout S-1.  Ends in layout 0.
template <int CF, bool G0, int A>
__device__ __forceinline__ void hunmix_group1(float2 (&v)[A], float2* xb, uint32_t tau, float t, uint32_t pm) {
    using H = HStages<CF, G0>;
    static_for<0, H::S>([&](auto J) {
        constexpr int st = H::S - 1 - decltype(J)::value;
        if constexpr (st < H::S - 1) hxpose<CF, H::rot(st + 1), H::rot(st)>(v, xb, tau);
        hmix<CF, H::rot(st), (st == H::S - 1 ? H::LB : -1), G0>(v, -t, pm);
    });
}

// Mixer of the dropped qubit k-1 between the two tiles of a pair (partner in the same
// register), and its undo on psi and lambda with the weighted share of Im <lambda|X|psi>.
template <int A>
__device__ __forceinline__ void hflip(float2 (&a)[A], float2 (&b)[A], float t) {
#pragma unroll
    for (int r = 0; r < A; ++r) bfly(a[r], b[r], t);
}
template <int A>
__device__ __forceinline__ float hunflip2(float2 (&fa)[A], float2 (&fb)[A], float2 (&la)[A], float2 (&lb)[A], float t,
                                          float k2, float& w) {
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        bfly(fa[r], fb[r], -t);
        bfly(la[r], lb[r], -t);
        if (r & 1) xacc(a1, la[r], lb[r], fa[r], fb[r]);
        else xacc(a0, la[r], lb[r], fa[r], fb[r]);
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    w *= k2;
    return w * (a0 + a1);
}

// Geometry of pass group grp over kh stored qubits: tile bit i -> global bit gmap(i).
__device__ __forceinline__ int hgroup_bits(int k, int grp, int i, int& h) {
    if (grp == 0) {
        h = HT;
        return i;
    }
    const int lo = HT + 9 * (grp - 1);
    h = min(k, lo + 9) - lo;
    if (i < h) return lo + i;
    if (i < 9) return 4 + (i - h);
    return i - 9;
}

// Block-wide sum in a fixed order (identical in every thread).
template <int W>
__device__ __forceinline__ double block_sum(double x, double* red) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W / 64; ++w) s += red[w];
    return s;
}

// Real weights: the cut value of every amplitude as a float, C - c0 = (k0 - c0) +
// sum_b q_b L_b + C_tt(q) with the coefficients summed in FP64 by one thread each (a fixed
// order), and its phase computed per amplitude (rphase).  cv(r) gives register r's value in
// layout 0.
template <int A, class CV>
__device__ __forceinline__ void gen_stage_cv(float2 (&f)[A], CV&& cv, double gpi, float sc) {
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 t = rphase(gpi, cv(r));
        f[r] = make_float2(sc * t.x, sc * t.y);
    }
}
template <int A, class CV>
__device__ __forceinline__ void phase_stage_cv(float2 (&f)[A], CV&& cv, double gpi, float sc) {
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 t = rphase(gpi, cv(r));
        f[r] = cmul(f[r], make_float2(sc * t.x, sc * t.y));
    }
}
template <bool UNDO, int A, class CV>
__device__ __forceinline__ float cgrad_stage_cv(float2 (&f)[A], float2 (&l)[A], CV&& cv, double gpi, float c0,
                                                float sc) {
    float a = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float c = cv(r);
        cacc(a, c + c0, l[r], f[r]);
        if constexpr (UNDO) {
            const float2 t0 = rphase(gpi, c);
            const float2 t = make_float2(sc * t0.x, sc * t0.y);
            f[r] = cmulc(f[r], t);
            l[r] = cmulc(l[r], t);
        }
    }
    return a;
}

// DB: two LDS buffers (psi and lambda transposed together) for the adjoint tile-pair
// passes, which run one workgroup per CU anyway (registers).  RW: real weights (one buffer).
template <int KIND, bool G0, bool DB = false, bool RW = false>
__global__ void __launch_bounds__((Hz<pass_cf(KIND, G0)>::W), (Hz<pass_cf(KIND, G0)>::WPE))
k_pass(PassArgs pa) {
    constexpr int CF = pass_cf(KIND, G0);
    constexpr bool GR = KIND >= GR_GEN_FINAL;
    constexpr bool PAIR = CF >= 2;
    constexpr int NT = PAIR ? 2 : 1;                       // tiles held at once
    using H = Hz<CF>;
    using HS = HStages<CF, G0>;
    constexpr int A = H::A;
    constexpr int NW = (A + 3) / 4;
    constexpr bool FINAL = (KIND == FWD_GEN_FINAL || KIND == FWD_BND_FINAL || KIND == GR_GEN_FINAL ||
                            KIND == GR_BND_FINAL);
    constexpr bool CUTS = !(KIND == FWD_MIX || KIND == RV_MIX);   // phases or C inner products
    __shared__ float2 xbuf[(DB ? 2 : 1) * H::NPAD];
    __shared__ __attribute__((aligned(16))) uint8_t ttl[RW ? 4 * HN : HN];   // C_tt: bytes, or floats (RW)
    __shared__ int32_t lcoef[NT][HT];
    __shared__ float lcf[RW ? NT : 1][HT + 1];   // RW: L_b and k0 - c0 of the unit's tiles
    __shared__ double red[H::W / 64];
    __shared__ int32_t k0_sh[NT];
    __shared__ int8_t tpos[32];          // tile bit of each global bit, -1 outside the tile
    extern __shared__ float2 rows[];   // [3][rowcap]

    const int tid = threadIdx.x;
    const uint32_t tau = static_cast<uint32_t>(tid);
    const int k = pa.k, kh = pa.kh;
    const int64_t tiles = int64_t{1} << (kh - HT);
    const int64_t units = PAIR ? tiles / 2 : tiles;       // tiles or tile pairs per item
    const int64_t wpi = units / pa.tpw;                   // workgroups per item
    const int64_t bslot = blockIdx.x / wpi;               // item within the batch
    const int64_t unit0 = (blockIdx.x - bslot * wpi) * pa.tpw;
    const int64_t item = pa.item0 + bslot;
    const int P = pa.ea.P, p = pa.ea.p;
    const int64_t cslot = item / P;
    const int point = static_cast<int>(item - cslot * P);
    const ConeHbm cd = pa.cones[cslot];

    // ---- per-item set-up: group geometry, C_tt table, phase rows
    int h = 0;
    uint32_t tmask = 0;  // global bits inside the tile
    for (int i = 0; i < HT; ++i) tmask |= 1u << hgroup_bits(kh, pa.group, i, h);
    const uint32_t pm = (pa.group == 0) ? (HN - 1u) : ((1u << h) - 1u);
    const int32_t k0_base = pa.cones[cslot].tt_min[pa.group] - cd.cut_min;
    if (CUTS && tid < 32) tpos[tid] = -1;
    // the phase rows a pass reads -> LDS: [0] layer 1, [1] layer lb, [2] layer p
    const size_t ipt = static_cast<size_t>(cd.inst) * P + point;   // angle point of the cone's instance
    const float2* ph0 = pa.ea.phase + ipt * p * pa.ea.R + cd.cut_shift;
    const float2* row_first = rows;
    const float2* row_lb = rows + pa.rowcap;
    const float2* row_last = rows + 2 * pa.rowcap;
    if constexpr (CUTS && RW) {
        const float* src = reinterpret_cast<const float*>(pa.tt) + pa.cones[cslot].tt_off[pa.group];
        for (uint32_t q = tau * 4; q < HN; q += H::W * 4)
            *reinterpret_cast<float4*>(reinterpret_cast<float*>(ttl) + q) = *reinterpret_cast<const float4*>(src + q);
    } else if constexpr (CUTS) {
        const uint8_t* src = pa.tt + pa.cones[cslot].tt_off[pa.group];
        for (uint32_t q = tau * 16; q < HN; q += H::W * 16)
            *reinterpret_cast<uint4*>(ttl + q) = *reinterpret_cast<const uint4*>(src + q);
        const int lsel[3] = {0, pa.lb > 0 ? pa.lb - 1 : 0, p - 1};
#pragma unroll
        for (int s = 0; s < 3; ++s)
            for (int c = tid; c < cd.cut_range; c += H::W)
                rows[s * pa.rowcap + c] = ph0[static_cast<size_t>(lsel[s]) * pa.ea.R + c];
    }
    __syncthreads();
    if (CUTS && tid < HT) {
        int hh;
        tpos[hgroup_bits(kh, pa.group, tid, hh)] = static_cast<int8_t>(tid);
    }
    // the thread's first cone edge, kept in registers for every tile
    int e0a = 0, e0b = 0, e0w = 0;
    if (CUTS && tid < cd.n_edges) {
        e0a = pa.e_a[cd.edge_off + tid];
        e0b = pa.e_b[cd.edge_off + tid];
        e0w = pa.e_w[cd.edge_off + tid];
    }

    // ---- global addressing of the I/O layout.  The global bit of every tile bit depends
    // only on (kh, group), so the per-register offsets are uniform (scalar registers); only
    // the thread's own offset lives in a vector register.
    constexpr int RIO = HS::IO;
    constexpr uint32_t TBITS_IO = rotl13(static_cast<uint32_t>(H::W - 1) << H::AB, RIO);  // thread bits
    constexpr uint32_t TBITS_0 = static_cast<uint32_t>(H::W - 1) << H::AB;                // same, layout 0
    uint32_t gbit[HT];
#pragma unroll
    for (int i = 0; i < HT; ++i) {
        int hh;
        gbit[i] = static_cast<uint32_t>(hgroup_bits(kh, pa.group, i, hh));
    }
    const uint32_t qio = htbase<CF, RIO>(tau);
    // the thread's byte offsets (its own tile coordinates, and complemented ones for the
    // second tile of a pair): its bits sit at most at global bit 26 (group 0: 12), so they
    // fit 32 bits and the loads use a scalar base plus a 32-bit vector offset
    uint32_t tbyte = 0, tbyte_c = 0;
#pragma unroll
    for (int i = 0; i < HT; ++i) {
        if ((qio >> i) & 1u) tbyte += 8u << gbit[i];
        if ((~qio & TBITS_IO) >> i & 1u) tbyte_c += 8u << gbit[i];
    }
    auto io_off = [&](int r) -> uint64_t {
        uint64_t o = 0;
        const uint32_t q = hroff<CF, RIO>(r);
#pragma unroll
        for (int i = 0; i < HT; ++i)
            if ((q >> i) & 1u) o += uint64_t{1} << gbit[i];
        return o;
    };
    // tile t of the unit: t = 0 in its own coordinates, t = 1 (pairs) complemented: register
    // r of thread tau holds local index ~q(tau, r) = (complemented thread bits) | roff(A-1-r).
    // (The thread offset is made opaque at every use so that no per-register address is
    // computed ahead and held in vector registers.)
    auto load = [&](float2 (&v)[A], const float2* buf, size_t off, int t) {
        const uint32_t tb = opaque_u32(t ? tbyte_c : tbyte);
#pragma unroll
        for (int r = 0; r < A; ++r)
            v[r] = *reinterpret_cast<const float2*>(
                reinterpret_cast<const char*>(buf + off + io_off(t ? A - 1 - r : r)) + tb);
    };
    auto store = [&](const float2 (&v)[A], float2* buf, size_t off, int t) {
        const uint32_t tb = opaque_u32(t ? tbyte_c : tbyte);
#pragma unroll
        for (int r = 0; r < A; ++r)
            *reinterpret_cast<float2*>(reinterpret_cast<char*>(buf + off + io_off(t ? A - 1 - r : r)) + tb) = v[r];
    };
    // prefetch: the next unit's psi (and, reverse passes, lambda) while this unit is worked on
    constexpr bool PF = pass_pf(KIND, G0);
    constexpr int NPF = (KIND == RV_MIX || KIND == RV_BND_MIX) ? 2 : 1;
    float2 nx[PF ? NPF : 1][PF ? NT : 1][PF ? A : 1];
    (void)nx;
    float2* xb = xbuf;
    float2* xb2 = DB ? xbuf + H::NPAD : nullptr;
    const float2* mix0 = pa.ea.mix + ipt * p;
    auto kpowK = [&](float k2) { return exp2f(0.5f * k * log2f(k2)); };
    // the angle-table entries the pass uses, read once (reads inside the unit loop would be
    // vector loads queued behind the prefetched states)
    auto mix_at = [&](int l) { return mix0[l < 1 ? 0 : (l > p ? p - 1 : l - 1)]; };
    const float2 mxa = mix_at(pa.la), mxb = mix_at(pa.lb), mx1 = mix0[0], mxp = mix0[p - 1];
    const float2 mxf = mix_at(pa.fix_layer);
    const float k2p = mxp.y;
    constexpr int RL = HS::rot(HS::S - 1);   // last processing layout

    // Per-thread partial sums over the workgroup's tiles, reduced once at the end into the
    // slot of (item, first unit): [0] = zz, [1 + l - 1] = d/d gamma_l, [1 + p + l - 1] =
    // d/d beta_l.  Which partial goes to which slot depends on the pass kind.
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    int slot[4] = {-1, -1, -1, -1};
    if constexpr (KIND == FWD_GEN_FINAL || KIND == FWD_BND_FINAL) {
        slot[0] = 0;
    } else if constexpr (KIND == GR_GEN_FINAL) {
        slot[0] = 0; slot[1] = 2 * p; slot[2] = 1;
    } else if constexpr (KIND == GR_BND_FINAL) {
        slot[0] = 0; slot[1] = 2 * p; slot[2] = p; slot[3] = p + pa.la;
    } else if constexpr (KIND == RV_MIX) {
        slot[0] = p + pa.la;
    } else if constexpr (KIND == RV_GEN_MIX) {
        slot[0] = p + pa.lb; slot[1] = 1;
    } else if constexpr (KIND == RV_BND_MIX) {
        slot[0] = p + pa.lb; slot[1] = pa.lb; slot[2] = p + pa.la;
    }

    auto outer_of = [&](int64_t tile) {
        uint64_t x = 0;
        int64_t o = tile;
        for (int b = 0; b < kh; ++b)
            if (!((tmask >> b) & 1u)) {
                x |= static_cast<uint64_t>(o & 1) << b;
                o >>= 1;
            }
        return x;
    };
    // Outer bits of the units' tiles.  A workgroup's units are consecutive, so after the first
    // the outer bits follow by a masked increment (tile u + 1) or decrement (the complemented
    // tile of a pair, tiles - 1 - u, counts down) over the outer-bit mask: two scalar
    // operations instead of a loop over the stored bits.
    const uint64_t omask = ((uint64_t{1} << kh) - 1u) & ~static_cast<uint64_t>(tmask);
    uint64_t xnext[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) xnext[t] = outer_of(t ? tiles - 1 - unit0 : unit0);
    auto next_off = [&](int t) { return (static_cast<size_t>(bslot) << kh) + xnext[t]; };
    (void)next_off;

    // the first unit's states, loaded while the workgroup sets up its first unit; every unit
    // takes its states from the prefetch registers, so no working register waits on a load
    if constexpr (PF) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            load(nx[0][t], pa.phi_in, next_off(t), t);
            if constexpr (NPF == 2) load(nx[NPF - 1][t], pa.lam, next_off(t), t);
        }
    }
    for (int64_t unit = unit0; unit < unit0 + pa.tpw; ++unit) {
        // ---- outer bits of the unit's tiles and their linear cut coefficients: an edge
        // between tile bit b and an outer bit o adds w (1 - 2 x_o) to lcoef[b] and w x_o to
        // k0; an edge between two outer bits adds w (x_o1 xor x_o2) to k0 (integer atomics:
        // exact in any order).  Qubit k-1 is an outer bit fixed at 0.
        uint64_t xo[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) xo[t] = xnext[t];
        xnext[0] = ((xnext[0] | ~omask) + 1u) & omask;
        if constexpr (NT > 1) xnext[1] = (xnext[1] - 1u) & omask;
        uint32_t pk[NT][NW];
        // real weights: the thread's base value, the register-bit coefficients and the
        // thread bits of each tile in layout 0
        float lthrf[NT], lcr[NT][H::AB];
        uint32_t qbt[NT];
        const float* ttf = reinterpret_cast<const float*>(ttl);
        if constexpr (CUTS && RW) {
            __syncthreads();   // the previous unit has read lcf
            if (tid < NT * (HT + 1)) {
                // coefficient b of tile t (b = HT: the constant, minus c0), summed in FP64 over
                // the cone's edges in their order
                const int t = tid / (HT + 1), b = tid - t * (HT + 1);
                const uint64_t x = xo[t];
                double acc = 0.0;
                for (int e = 0; e < cd.n_edges; ++e) {
                    const int ea_ = pa.e_a[cd.edge_off + e], eb_ = pa.e_b[cd.edge_off + e];
                    const double w = pa.e_wd[cd.edge_off + e];
                    const int ia = tpos[ea_], ib = tpos[eb_];
                    const int xa = static_cast<int>((x >> ea_) & 1u), xb = static_cast<int>((x >> eb_) & 1u);
                    if (b < HT) {
                        if (ia == b && ib < 0) acc += xb ? -w : w;
                        else if (ib == b && ia < 0) acc += xa ? -w : w;
                    } else if (ia >= 0 && ib < 0) {
                        if (xb) acc += w;
                    } else if (ia < 0 && ib >= 0) {
                        if (xa) acc += w;
                    } else if (ia < 0 && ib < 0 && (xa ^ xb)) {
                        acc += w;
                    }
                }
                lcf[t][b] = b < HT ? static_cast<float>(acc) : static_cast<float>(acc - static_cast<double>(cd.c0));
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                qbt[t] = t ? (~htbase<CF, 0>(tau) & TBITS_0) : htbase<CF, 0>(tau);
                float c = lcf[t][HT];
#pragma unroll
                for (int i = H::AB; i < HT; ++i)
                    if ((qbt[t] >> i) & 1u) c += lcf[t][i];
                lthrf[t] = c;
#pragma unroll
                for (int i = 0; i < H::AB; ++i) lcr[t][i] = lcf[t][i];
            }
        } else if constexpr (CUTS) {
            __syncthreads();   // the previous unit has read lcoef and k0
            if (tid < HT) {
#pragma unroll
                for (int t = 0; t < NT; ++t) lcoef[t][tid] = 0;
            }
            if (tid == 0) {
#pragma unroll
                for (int t = 0; t < NT; ++t) k0_sh[t] = k0_base;
            }
            __syncthreads();
            auto add_edge = [&](int a, int b, int w) {
                const int ia = tpos[a], ib = tpos[b];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int xa = static_cast<int>((xo[t] >> a) & 1u), xb2 = static_cast<int>((xo[t] >> b) & 1u);
                    if (ia >= 0 && ib < 0) {
                        atomicAdd(&lcoef[t][ia], w - 2 * w * xb2);
                        if (xb2) atomicAdd(&k0_sh[t], w);
                    } else if (ia < 0 && ib >= 0) {
                        atomicAdd(&lcoef[t][ib], w - 2 * w * xa);
                        if (xa) atomicAdd(&k0_sh[t], w);
                    } else if (ia < 0 && ib < 0 && (xa ^ xb2)) {
                        atomicAdd(&k0_sh[t], w);
                    }
                }
            };
            if (tid < cd.n_edges) add_edge(e0a, e0b, e0w);
            for (int e = tid + H::W; e < cd.n_edges; e += H::W)
                add_edge(pa.e_a[cd.edge_off + e], pa.e_b[cd.edge_off + e], pa.e_w[cd.edge_off + e]);
            __syncthreads();

            // packed cut values (minus cut_min) of the thread's amplitudes in layout rotation 0
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const uint32_t qb = t ? (~htbase<CF, 0>(tau) & TBITS_0) : htbase<CF, 0>(tau);
                int32_t lthr = k0_sh[t];
#pragma unroll
                for (int i = 0; i < HT; ++i)
                    if ((qb >> i) & 1u) lthr += lcoef[t][i];
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) pk[t][w2] = 0u;
#pragma unroll
                for (int r = 0; r < A; ++r) {
                    const int rr = t ? A - 1 - r : r;
                    int32_t c = lthr + ttl[qb | hroff<CF, 0>(rr)];
#pragma unroll
                    for (int i = 0; i < H::AB; ++i)
                        if ((rr >> i) & 1) c += lcoef[t][i];
                    pk[t][r >> 2] |= static_cast<uint32_t>(c) << (8 * (r & 3));
                }
            }
        }
        // register r of tile t (layout 0): its real cut value minus c0
        auto CV = [&](int t) {
            return [&, t](int r) {
                const int rr = t ? A - 1 - r : r;
                float c = lthrf[t] + ttf[qbt[t] | hroff<CF, 0>(rr)];
#pragma unroll
                for (int i = 0; i < H::AB; ++i)
                    if ((rr >> i) & 1) c += lcr[t][i];
                return c;
            };
        };
        const double* gam = RW ? pa.ea.gamma + (static_cast<size_t>(cd.inst) * pa.ea.gamma_P + point) * p : nullptr;
        auto GPI = [&](int l) { return gam[l] * 0.31830988618379067154; };   // gamma_(l+1) / pi
        (void)CV;
        (void)GPI;
        size_t off[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) off[t] = (static_cast<size_t>(bslot) << kh) + xo[t];

        float2 f[NT][A];
        // ------------------------------------------------------------ forward part
        if constexpr (KIND == FWD_GEN_MIX || KIND == FWD_GEN_FINAL || KIND == GR_GEN_FINAL) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if constexpr (RW) gen_stage_cv(f[t], CV(t), GPI(0), exp2f(-0.5f * k) * (p == 1 ? k2p : 1.f));
                else gen_stage(f[t], pk[t], row_first, exp2f(-0.5f * k) * (p == 1 ? k2p : 1.f));
            }
            if constexpr (KIND == FWD_GEN_MIX) {
                const float t1 = mx1.x;
#pragma unroll
                for (int t = 0; t < NT; ++t) hmix_group<CF, G0, false, 0>(f[t], xb, tau, t1, pm);
                if constexpr (PAIR) hflip(f[0], f[1], t1);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    hxpose<CF, RL, RIO>(f[t], xb, tau);
                    store(f[t], pa.phi, off[t], t);
                }
                continue;
            }
        }
        if constexpr (KIND == FWD_MIX || KIND == FWD_BND_MIX || KIND == FWD_BND_FINAL || KIND == GR_BND_FINAL) {
            if constexpr (PF) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < A; ++r) f[t][r] = nx[0][t][r];
                if (unit + 1 < unit0 + pa.tpw) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) load(nx[0][t], pa.phi_in, next_off(t), t);
                }
            } else {
#pragma unroll
                for (int t = 0; t < NT; ++t) load(f[t], pa.phi_in, off[t], t);
            }
            const float2 tka = mxa;
#pragma unroll
            for (int t = 0; t < NT; ++t) hmix_group<CF, G0, true, RIO>(f[t], xb, tau, tka.x, pm);   // ends in rotation 0
            if constexpr (PAIR) hflip(f[0], f[1], tka.x);
            if constexpr (KIND == FWD_MIX) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    hxpose<CF, 0, RIO>(f[t], xb, tau);
                    store(f[t], pa.phi, off[t], t);
                }
                continue;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if constexpr (RW) phase_stage_cv(f[t], CV(t), GPI(pa.lb - 1), kpowK(tka.y) * (pa.lb == p ? k2p : 1.f));
                else phase_stage(f[t], pk[t], row_lb, kpowK(tka.y) * (pa.lb == p ? k2p : 1.f));
            }
            if constexpr (KIND == FWD_BND_MIX) {
                const float tb = mxb.x;
#pragma unroll
                for (int t = 0; t < NT; ++t) hmix_group<CF, G0, false, 0>(f[t], xb, tau, tb, pm);
                if constexpr (PAIR) hflip(f[0], f[1], tb);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    hxpose<CF, RL, RIO>(f[t], xb, tau);
                    store(f[t], pa.phi, off[t], t);
                }
                continue;
            }
        }
        // ------------------------------------------------------------ final layer
        if constexpr (FINAL) {
            const float tp = mxp.x;
            double zzp = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
#pragma unroll
                for (int r = 0; r < A; ++r)
                    if (!(r & 1)) bfly(f[t][r], f[t][r | 1], tp);
#pragma unroll
                for (int r = 0; r < A; ++r)
                    if (!(r & 2)) bfly(f[t][r], f[t][r | 2], tp);
#pragma unroll
                for (int r = 0; r < A; ++r) {
                    const double pr = static_cast<double>(fmaf(f[t][r].x, f[t][r].x, f[t][r].y * f[t][r].y));
                    zzp += (((r ^ (r >> 1)) & 1) ? -pr : pr);
                }
            }
            part[0] += zzp;
            if constexpr (GR) {
                float2 lm[NT][A];
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
#pragma unroll
                    for (int r = 0; r < A; ++r)
                        lm[t][r] = (((r ^ (r >> 1)) & 1) ? make_float2(-f[t][r].x, -f[t][r].y) : f[t][r]);
#pragma unroll
                    for (int r = 0; r < A; ++r)
                        if (!(r & 1)) xacc(acc, lm[t][r], lm[t][r | 1], f[t][r], f[t][r | 1]);
#pragma unroll
                    for (int r = 0; r < A; ++r)
                        if (!(r & 2)) xacc(acc, lm[t][r], lm[t][r | 2], f[t][r], f[t][r | 2]);
#pragma unroll
                    for (int r = 0; r < A; ++r)
                        if (!(r & 2)) { bfly(f[t][r], f[t][r | 2], -tp); bfly(lm[t][r], lm[t][r | 2], -tp); }
#pragma unroll
                    for (int r = 0; r < A; ++r)
                        if (!(r & 1)) { bfly(f[t][r], f[t][r | 1], -tp); bfly(lm[t][r], lm[t][r | 1], -tp); }
                }
                part[1] += 2.0 * static_cast<double>(acc);
                const float mu = k2p;
                if constexpr (KIND == GR_GEN_FINAL) {
                    float a = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if constexpr (RW) a += cgrad_stage_cv<false>(f[t], lm[t], CV(t), 0.0, cd.c0, 1.f);
                        else a += cgrad_stage<false>(f[t], lm[t], pk[t], row_first, cd.cut_min, 1.f);
                    }
                    part[2] += 2.0 * static_cast<double>(mu) * mu * a;
                } else {
                    float a = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if constexpr (RW) a += cgrad_stage_cv<true>(f[t], lm[t], CV(t), GPI(p - 1), cd.c0, mu);
                        else a += cgrad_stage<true>(f[t], lm[t], pk[t], row_last, cd.cut_min, mu);
                    }
                    part[2] += 2.0 * static_cast<double>(mu) * mu * a;
                    // mixer la = p-1 on this group: psi is not needed after this pass (the next
                    // reverse pass reads it from device memory), so the inner products of all
                    // the group's qubits are taken at this point of the layer (both states
                    // at the scale |kappa|^-m0a: weight |kappa|^2m0a), and only lambda is
                    // then undone
                    const float2 tka = mxa;
                    const float w0 = exp2f(pa.m0a * log2f(tka.y));
                    float b = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) b += hip_group<CF, G0, DB>(f[t], lm[t], xb, tau, pm, xb2);
                    if constexpr (PAIR) {
                        float a0 = 0.f, a1 = 0.f;
#pragma unroll
                        for (int r = 0; r < A; ++r) {
                            if (r & 1) xacc(a1, lm[0][r], lm[1][r], f[0][r], f[1][r]);
                            else xacc(a0, lm[0][r], lm[1][r], f[0][r], f[1][r]);
                            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                        }
                        b += a0 + a1;
                        hflip(lm[0], lm[1], -tka.x);
                    }
                    part[3] += 2.0 * static_cast<double>(w0) * static_cast<double>(b);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        hunmix_group1<CF, G0>(lm[t], xb, tau, tka.x, pm);
                        hxpose<CF, 0, RIO>(lm[t], xb, tau);
                        store(lm[t], pa.lam, off[t], t);
                    }
                }
            }
        }
        // ------------------------------------------------------------ reverse passes
        if constexpr (KIND == RV_GEN_MIX) {
            // The undo of the first forward pass (group lb of layer 1, lb = 1): psi there is
            // D_1 |+> mixed by this group, so it is neither loaded nor undone.  lambda alone is
            // undone; D_1 |+> is regenerated from the cut values, and every term of this pass
            // (the group's beta_1 inner products, the dropped qubit's with pairs, and gamma_1)
            // is taken at that point, the start of layer 1 (X_j commutes with every mixer of
            // its layer).  Layer 1 is then undone completely, so lambda carries 1/mu_1
            // (mu_1 = |kappa_1|^k) and psi_0 its true norm: weight mu_1.
            float2 lm[NT][A];
#pragma unroll
            for (int t = 0; t < NT; ++t) load(lm[t], pa.lam, off[t], t);
            const float2 tkb = mxb;
#pragma unroll
            for (int t = 0; t < NT; ++t) hmix_group<CF, G0, true, RIO>(lm[t], xb, tau, -tkb.x, pm);   // ends in layout 0
            if constexpr (PAIR) hflip(lm[0], lm[1], -tkb.x);
            const float mu = kpowK(tkb.y);
            const float sc = exp2f(-0.5f * k);
            // D_1 |+> of tile t, register r (layout 0)
            auto psi0 = [&](int t, int r) {
                if constexpr (RW) {
                    const float2 v = rphase(GPI(0), CV(t)(r));
                    return make_float2(sc * v.x, sc * v.y);
                } else {
                    const float2 v = row_first[cutv<A>(pk[t], r)];
                    return make_float2(sc * v.x, sc * v.y);
                }
            };
            float a = 0.f, b = 0.f;
            if constexpr (PAIR) {
                float b0 = 0.f, b1 = 0.f;
#pragma unroll
                for (int r = 0; r < A; ++r) {
                    if (r & 1) xacc(b1, lm[0][r], lm[1][r], psi0(0, r), psi0(1, r));
                    else xacc(b0, lm[0][r], lm[1][r], psi0(0, r), psi0(1, r));
                    if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
                b = b0 + b1;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
#pragma unroll
                for (int r = 0; r < A; ++r) f[t][r] = psi0(t, r);
                if constexpr (RW) a += cgrad_stage_cv<false>(f[t], lm[t], CV(t), 0.0, cd.c0, 1.f);
                else a += cgrad_stage<false>(f[t], lm[t], pk[t], row_first, cd.cut_min, 1.f);
                b += hip_group<CF, G0, DB>(f[t], lm[t], xb, tau, pm, xb2);
            }
            part[0] += 2.0 * static_cast<double>(mu) * static_cast<double>(b);
            part[1] += 2.0 * static_cast<double>(mu) * static_cast<double>(a);
        }
        if constexpr (KIND == RV_MIX || KIND == RV_BND_MIX) {
            float2 lm[NT][A];
            if constexpr (PF) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < A; ++r) {
                        f[t][r] = nx[0][t][r];
                        lm[t][r] = nx[1][t][r];
                    }
                if (unit + 1 < unit0 + pa.tpw) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const size_t o = next_off(t);
                        load(nx[0][t], pa.phi_in, o, t);
                        load(nx[1][t], pa.lam, o, t);
                    }
                }
            } else {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    load(f[t], pa.phi_in, off[t], t);
                    load(lm[t], pa.lam, off[t], t);
                }
            }
            if (pa.fix_layer > 0) {
                // psi read as the forward sweep left it (the first reverse pass, or every reverse
                // pass reading a stored checkpoint) carries the factored mixer's scale of the
                // forward direction, 1/|kappa_l| per qubit of the layer l in progress mixed so
                // far (m of them), where lambda carries 1/|kappa_l| per qubit of that layer
                // undone (k - m): psi is rescaled by |kappa_l|^(2m - k) (host: fix_pow).  For
                // the first reverse pass of the uncompute program m = k - 14.
                const float sc = exp2f(0.5f * pa.fix_pow * log2f(mxf.y));
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int r = 0; r < A; ++r) f[t][r] = make_float2(sc * f[t][r].x, sc * f[t][r].y);
            }
            if constexpr (KIND == RV_MIX) {
                const float2 tka = mxa;
                const float w0 = exp2f(pa.m0a * log2f(tka.y));
                float w = w0, b = 0.f;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    w = w0;
                    b += hunmix_group<CF, G0, true, RIO, DB>(f[t], lm[t], xb, tau, tka.x, tka.y, w, pm, xb2);
                }
                if constexpr (PAIR) b += hunflip2(f[0], f[1], lm[0], lm[1], tka.x, tka.y, w);
                part[0] += 2.0 * static_cast<double>(b);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (pa.store_phi) {
                        if constexpr (DB) {
                            hxpose_dual<CF, 0, RIO>(f[t], lm[t], xb, xb2, tau);
                        } else {
                            hxpose<CF, 0, RIO>(f[t], xb, tau);
                            hxpose<CF, 0, RIO>(lm[t], xb, tau);
                        }
                        store(f[t], pa.phi, off[t], t);
                    } else {
                        hxpose<CF, 0, RIO>(lm[t], xb, tau);
                    }
                    store(lm[t], pa.lam, off[t], t);
                }
            } else {
                // undo mixer lb (the first group of layer lb in forward order: after it, layer
                // lb is completely undone), then gamma_lb
                const float2 tkb = mxb;
                const float w0 = exp2f(pa.m0b * log2f(tkb.y));
                float w = w0, b = 0.f;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    w = w0;
                    b += hunmix_group<CF, G0, true, RIO, DB>(f[t], lm[t], xb, tau, tkb.x, tkb.y, w, pm, xb2);
                }
                if constexpr (PAIR) b += hunflip2(f[0], f[1], lm[0], lm[1], tkb.x, tkb.y, w);
                part[0] += 2.0 * static_cast<double>(b);
                const float mu = (pa.lb == p) ? k2p : kpowK(tkb.y);
                {
                    float a = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if constexpr (RW) a += cgrad_stage_cv<true>(f[t], lm[t], CV(t), GPI(pa.lb - 1), cd.c0, mu);
                        else a += cgrad_stage<true>(f[t], lm[t], pk[t], row_lb, cd.cut_min, mu);
                    }
                    part[1] += 2.0 * static_cast<double>(mu) * mu * a;
                    const float2 tka = mxa;
                    const float wa0 = exp2f(pa.m0a * log2f(tka.y));
                    float wa = wa0, ba = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        wa = wa0;
                        ba += hunmix_group<CF, G0, false, 0, DB>(f[t], lm[t], xb, tau, tka.x, tka.y, wa, pm, xb2);
                    }
                    if constexpr (PAIR) ba += hunflip2(f[0], f[1], lm[0], lm[1], tka.x, tka.y, wa);
                    part[2] += 2.0 * static_cast<double>(ba);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if (pa.store_phi) {
                            if constexpr (DB) {
                                hxpose_dual<CF, RL, RIO>(f[t], lm[t], xb, xb2, tau);
                            } else {
                                hxpose<CF, RL, RIO>(f[t], xb, tau);
                                hxpose<CF, RL, RIO>(lm[t], xb, tau);
                            }
                            store(f[t], pa.phi, off[t], t);
                        } else {
                            hxpose<CF, RL, RIO>(lm[t], xb, tau);
                        }
                        store(lm[t], pa.lam, off[t], t);
                    }
                }
            }
        }
    }
    double* gp = pa.gpart + (static_cast<size_t>(bslot) * tiles + unit0) * (2 * p + 1);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (slot[i] >= 0) {
            const double t = block_sum<H::W>(part[i], red);
            if (tid == 0) gp[slot[i]] += t;
        }
}

}  // namespace qaoa

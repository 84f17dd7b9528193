// Workgroup-resident light-cone kernel: one (cone, angle point) item is simulated
// entirely inside a workgroup, forward and (optionally) adjoint, for cones of up to 14
// qubits.
//
// State layout.  An item's 2^K complex64 amplitudes are spread over TPI threads with
// A = 2^AB amplitudes each in registers.  In "stage" st the amplitude held by thread
// tau in register r has basis index q = rotl_K((tau << AB) | r, st * AB): the AB
// register bits cover qubits st*AB .. st*AB+AB-1, so the single-qubit mixers of those
// qubits are butterflies between registers.  Moving between stages is a transpose
// through LDS (padded against bank conflicts).  Layers alternate the stage order
// so that consecutive layers share a stage and the last full layer ends in stage 0,
// which holds qubits 0 and 1 (u and v) for the final two-qubit mixer and <Z_0 Z_1>.
//
// Steps (Sec. 2.2 ansatz with the MaxCut cost of Sec. 2.4, on the cone of Sec. 2.3):
//   psi = 2^{-K/2} exp(-i gamma_1 C(x))                 (|+>^K then U_P(gamma_1))
//   for l = 1..p-1: mixer exp(-i beta_l X_j) on every qubit, then exp(-i gamma_{l+1} C)
//   last layer: mixer on qubits 0 and 1 only (the others commute through Z_0 Z_1)
//   zz = sum_x |psi_x|^2 (1 - 2 (x_0 xor x_1)), accumulated in FP64
// Adjoint (GRAD): lambda = Z_0 Z_1 psi, then the layers are undone in reverse on both
// psi and lambda, with
//   d zz / d beta_l  = 2 Im <lambda| sum_j X_j |psi>   (taken while undoing mixer l)
//   d zz / d gamma_l = 2 Im <lambda| C |psi>          (after mixer l is undone)
// The forward state is recovered by the inverse layers, not stored.
//
// Global-flip halving (K >= 3): |+>, C(x) and every mixer are invariant under flipping all
// K qubits, so psi_x = psi_(x xor 1...1) and the same holds for lambda = Z_0 Z_1 psi.  Only
// the half with qubit K-1 = 0 is kept (the layout above is applied to K-1 qubits); the
// mixer of qubit K-1 pairs a stored amplitude with the complement of its index over the
// stored bits, and every sum over the half is doubled.
#pragma once

#include "device.hpp"

#include <algorithm>
#include <atomic>
#include <type_traits>

namespace qaoa {

// G bit 0 = 1 for the adjoint kernels, which hold two states and use 16 amplitudes per
// thread; G >> 1 selects a layout variant for the run-time tuner:
//   0  the default: 5 register bits per stage forward, 4 adjoint; workgroups of >= 64 threads
//   1  one register bit fewer per stage (qubits per LDS pass): more threads per item
//   2  workgroups of >= 256 threads (more cones per workgroup for small cones)
//   3  the 14-qubit adjoint kernel in the exchange layouts (one LDS transpose per layer)
#ifndef QAOA_FUSED_AB_GRAD
#define QAOA_FUSED_AB_GRAD 4
#endif
template <int K, int G = 0>
struct Fz {
    static constexpr int VAR = G >> 1;
    static constexpr int AB_MAX = ((G & 1) ? QAOA_FUSED_AB_GRAD : 5) - (VAR == 1 ? 1 : 0);
    static constexpr int AB = K < AB_MAX ? K : AB_MAX;  // register bits
    static constexpr int A = 1 << AB;              // amplitudes per thread per state
    static constexpr int TB = K - AB;              // thread bits per item
    static constexpr int TPI = 1 << TB;            // threads per item
    static constexpr int WGMIN = VAR == 2 ? 256 : 64;
    static constexpr int WG = TPI > WGMIN ? TPI : WGMIN;
    static constexpr int IPW = WG / TPI;           // items per workgroup
    // LQ: K = S * AB + 1, so the one qubit left over (K-1) sits on lane bit 0 in the last
    // stage and is mixed across lanes there instead of costing a stage of its own.
    static constexpr bool LQ = K % AB == 1 && K / AB >= 2;
    static constexpr int S = LQ ? K / AB : (K + AB - 1) / AB;   // stages
    static constexpr uint32_t N = 1u << K;
    static constexpr uint32_t NPAD = N + (N >> 4) + (N >> 8) + (AB == 5 ? 2 : 8) * (N >> 12);  // padded item buffer
};

template <int K>
__device__ constexpr uint32_t rotl(uint32_t x, int s) {
    return s == 0 ? x : (((x << s) | (x >> (K - s))) & ((1u << K) - 1u));
}
template <int K, int G, int ST>
__device__ constexpr uint32_t roff(int r) { return rotl<K>(static_cast<uint32_t>(r), ST * Fz<K, G>::AB); }
template <int K, int G, int ST>
__device__ __forceinline__ uint32_t tbase(uint32_t tau) { return rotl<K>(tau << Fz<K, G>::AB, ST * Fz<K, G>::AB); }

// LDS padding against bank conflicts: one slot per 16 and per 256 entries, and c per 4096
// (c = 8 for 4 register bits per stage, 2 for 5).  With 8-byte entries the 16 lanes that
// share an LDS cycle then hit 16 distinct bank pairs in every register stage of the 13-bit
// layouts (lane bits on qubits 4-7, 8-11, 12 0 1 2 for AB = 4; 5-8, 10 11 12 0, 2-5 for
// AB = 5), including the complement partners of the flip transposes.  It is additive over
// indices with disjoint bits, so pad(base | off) = pad(base) + pad(off) and every register
// of a transpose is addressed by one base register plus an immediate.
template <int AB = 4>
__device__ constexpr uint32_t pad(uint32_t q) { return q + (q >> 4) + (q >> 8) + (AB == 5 ? 2u : 8u) * (q >> 12); }

// Factored single-qubit mixer.  exp(-i beta X) = kappa X^e (1 - i tau X) with
//   |cos beta| >= |sin beta|: kappa = cos beta,     e = 0, tau = tan beta
//   otherwise:                kappa = -i sin beta,  e = 1, tau = -cot beta,
// so |tau| <= 1 and the butterfly is psi'_x = psi_x - i tau psi_{x xor 2^j}: one FMA per
// output component.  A full layer multiplies the state by kappa^k X^(e k); every cone
// state is invariant under flipping all cone qubits (|+>, C(x) and the mixer are), so
// X^(k) acts as the identity, and the real factor |kappa|^k is folded into the next
// phase row.  Undoing a layer uses tau -> -tau and gains a factor 1/|kappa|^2 per qubit.
__device__ __forceinline__ void bfly(float2& a, float2& b, float t) {
    const float2 a0 = a, b0 = b;
    a.x = fmaf(t, b0.y, a0.x);
    a.y = fmaf(-t, b0.x, a0.y);
    b.x = fmaf(t, a0.y, b0.x);
    b.y = fmaf(-t, a0.x, b0.y);
}

// Accumulations into a single register are written as in-order FMAs.  Left to itself the
// compiler defers such a dependent chain past the following butterflies and then has to
// keep whole earlier generations of both states alive (hundreds of registers); pinning
// the chain next to the butterfly that produced its inputs keeps the states in place.
// acc += Im(conj(la) pb) + Im(conj(lb) pa)
__device__ __forceinline__ void xacc(float& acc, float2 la, float2 lb, float2 pa, float2 pb) {
    asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(acc) : "v"(la.x), "v"(pb.y));
    asm volatile("v_fma_f32 %0, -%1, %2, %0" : "+v"(acc) : "v"(la.y), "v"(pb.x));
    asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(acc) : "v"(lb.x), "v"(pa.y));
    asm volatile("v_fma_f32 %0, -%1, %2, %0" : "+v"(acc) : "v"(lb.y), "v"(pa.x));
}

// acc += c * Im(conj(l) f)
__device__ __forceinline__ void cacc(float& acc, float c, float2 l, float2 f) {
    float im;
    asm volatile("v_mul_f32 %0, %1, %2" : "=v"(im) : "v"(l.x), "v"(f.y));
    asm volatile("v_fma_f32 %0, -%1, %2, %0" : "+v"(im) : "v"(l.y), "v"(f.x));
    asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(acc) : "v"(c), "v"(im));
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

// The same amplitude in the neighbouring lane (lane xor 1): DPP quad_perm [1, 0, 3, 2].
__device__ __forceinline__ float2 lane_x1(float2 v) {
    return make_float2(__int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.x), 0xB1, 0xF, 0xF, true)),
                       __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.y), 0xB1, 0xF, 0xF, true)));
}

template <int K, int G, int ST, int A>
__device__ __forceinline__ void mix_stage(float2 (&v)[A], float t) {
    constexpr int AB = Fz<K, G>::AB;
    if constexpr (Fz<K, G>::LQ && ST == Fz<K, G>::S - 1) {
        // qubit K-1 on lane bit 0: the butterfly partner is the neighbouring lane
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 q = lane_x1(v[r]);
            v[r] = make_float2(fmaf(t, q.y, v[r].x), fmaf(-t, q.x, v[r].y));
            if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < AB; ++i) {
        if (ST * AB + i >= K) continue;  // wrapped bit: handled in stage 0
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

// Undo the mixer on the stage's qubits for psi and lambda; returns the stage's share of
// Im <lambda| sum_j X_j |psi>.  X_j commutes with its own rotation, so the pair's term is
// taken after the butterfly; every undone qubit scales each state by 1/|kappa| (their inner
// products by 1/|kappa|^2), which the running weight w (= |kappa|^{2m} after m qubits)
// compensates.
template <int K, int G, int ST, int A>
__device__ __forceinline__ float unmix_stage2(float2 (&f)[A], float2 (&l)[A], float t, float k2, float& w) {
    constexpr int AB = Fz<K, G>::AB;
    float acc = 0.f;
    if constexpr (Fz<K, G>::LQ && ST == Fz<K, G>::S - 1) {
        // qubit K-1 across lanes; its term is taken on the values before the undo, with
        // the weight before this qubit
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 fq = lane_x1(f[r]);
            const float2 lq = lane_x1(l[r]);
            cacc(a, 1.f, l[r], fq);
            f[r] = make_float2(fmaf(-t, fq.y, f[r].x), fmaf(t, fq.x, f[r].y));
            l[r] = make_float2(fmaf(-t, lq.y, l[r].x), fmaf(t, lq.x, l[r].y));
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        acc = w * a;
        w *= k2;
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < AB; ++i) {
        if (ST * AB + i >= K) continue;
        float a0 = 0.f, a1 = 0.f;
        int np = 0;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & (1 << i))) {
                const int r2 = r | (1 << i);
                bfly(f[r], f[r2], -t);
                bfly(l[r], l[r2], -t);
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

// Last stage of the undo of layer 1: psi is not needed after it (D_1 |+> is regenerated
// from the cut table), so every term of the stage is taken at its entry (X_j commutes with
// all rotations of its layer, so the entry point is as good as the point after X_j's own
// undo) with the entry weight w, and the mixer is undone on lambda alone.
template <int K, int G, int ST, int A>
__device__ __forceinline__ float unmix_stage_last(const float2 (&f)[A], float2 (&l)[A], float t, float w) {
    constexpr int AB = Fz<K, G>::AB;
    constexpr bool LANE = Fz<K, G>::LQ && ST == Fz<K, G>::S - 1;
    float a0 = 0.f, a1 = 0.f;
    if constexpr (LANE) {
#pragma unroll
        for (int r = 0; r < A; ++r) {
            if (r & 1) cacc(a1, 1.f, l[r], lane_x1(f[r]));
            else cacc(a0, 1.f, l[r], lane_x1(f[r]));
            if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < AB; ++i) {
        if (ST * AB + i >= K) continue;
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
    if constexpr (LANE) {
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 lq = lane_x1(l[r]);
            l[r] = make_float2(fmaf(-t, lq.y, l[r].x), fmaf(t, lq.x, l[r].y));
            if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < AB; ++i) {
        if (ST * AB + i >= K) continue;
        int nb = 0;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & (1 << i))) {
                bfly(l[r], l[r | (1 << i)], -t);
                if ((++nb & 7) == 0) __builtin_amdgcn_sched_barrier(0);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
    return w * (a0 + a1);
}

// The transpose bases are loop-invariant; an empty asm makes them opaque so that the
// compiler keeps one base register plus immediate offsets instead of hoisting one
// address register per amplitude out of the layer loops.
__device__ __forceinline__ uint32_t opaque_u32(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

template <int K, int G, int FROM, int TO, int A>
__device__ __forceinline__ void xpose(float2 (&v)[A], float2* xb, uint32_t tau) {
    float2* pf = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, FROM>(tau)));
    const float2* pt = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(tau)));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) pf[pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) v[r] = pt[pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
}


// Global-flip halving.  Every cone state is invariant under flipping all K qubits, so only
// the half with qubit K-1 = 0 is stored: amplitude y (K-1 bits) stands for both y and its
// complement over all K bits.  The mixer of qubit K-1 then pairs y with ybar = y xor
// (2^(K-1) - 1), the complement over the stored bits, which lives in thread ~tau, register
// A-1-r of the same layout.  These transposes apply that butterfly on the way through LDS.
template <int K, int G, int FROM, int TO, int A>
__device__ __forceinline__ void xpose_flip(float2 (&v)[A], float2* xb, uint32_t tau, float t) {
    constexpr uint32_t TM = Fz<K, G>::TPI - 1;
    float2* pf = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, FROM>(tau)));
    const float2* pt = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(tau)));
    const float2* pc = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(~tau & TM)));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) pf[pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 a = pt[pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
        const float2 b = pc[pad<Fz<K, G>::AB>(roff<K, G, TO>(A - 1 - r))];
        v[r] = make_float2(fmaf(t, b.y, a.x), fmaf(-t, b.x, a.y));
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
}

// Undo the flip-qubit butterfly on psi and lambda while transposing both.  Returns the
// thread's share of Im <lambda| X_(K-1) |psi> on the values before the undo (the undone
// pair differs from them by the factor 1/|kappa|^2, which the caller's weight accounts for).
template <int K, int G, int FROM, int TO, int A>
__device__ __forceinline__ float xpose2_unflip(float2 (&f)[A], float2 (&l)[A], float2* xb, uint32_t tau, float t) {
    constexpr uint32_t TM = Fz<K, G>::TPI - 1;
    float2* pf = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, FROM>(tau)));
    const float2* pt = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(tau)));
    const float2* pc = xb + opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(~tau & TM)));
    float2 fp[A];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) pf[pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = f[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        f[r] = pt[pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
        fp[r] = pc[pad<Fz<K, G>::AB>(roff<K, G, TO>(A - 1 - r))];
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) pf[pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = l[r];
    __syncthreads();
    float acc = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 lo = pt[pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
        const float2 lq = pc[pad<Fz<K, G>::AB>(roff<K, G, TO>(A - 1 - r))];
        cacc(acc, 1.f, lo, fp[r]);
        l[r] = make_float2(fmaf(-t, lq.y, lo.x), fmaf(t, lq.x, lo.y));
        f[r] = make_float2(fmaf(-t, fp[r].y, f[r].x), fmaf(t, fp[r].x, f[r].y));
        if ((r & 1) == 1) __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// Two-buffer forms for the adjoint kernels that run one workgroup per CU (registers limit
// them there, so LDS has room for a second buffer): psi and lambda go through LDS together,
// one barrier pair instead of two.
template <int K, int G, int FROM, int TO, int A>
__device__ __forceinline__ void xpose_dual(float2 (&f)[A], float2 (&l)[A], float2* xa, float2* xc, uint32_t tau) {
    const uint32_t of = opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, FROM>(tau)));
    const uint32_t ot = opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(tau)));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        xa[of + pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = f[r];
        xc[of + pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = l[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        f[r] = xa[ot + pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
        l[r] = xc[ot + pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
    }
}

template <int K, int G, int FROM, int TO, int A>
__device__ __forceinline__ float xpose2_unflip_dual(float2 (&f)[A], float2 (&l)[A], float2* xa, float2* xc,
                                                    uint32_t tau, float t) {
    constexpr uint32_t TM = Fz<K, G>::TPI - 1;
    const uint32_t of = opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, FROM>(tau)));
    const uint32_t ot = opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(tau)));
    const uint32_t oc = opaque_u32(pad<Fz<K, G>::AB>(tbase<K, G, TO>(~tau & TM)));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        xa[of + pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = f[r];
        xc[of + pad<Fz<K, G>::AB>(roff<K, G, FROM>(r))] = l[r];
    }
    __syncthreads();
    float acc = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 fo = xa[ot + pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
        const float2 fq = xa[oc + pad<Fz<K, G>::AB>(roff<K, G, TO>(A - 1 - r))];
        const float2 lo = xc[ot + pad<Fz<K, G>::AB>(roff<K, G, TO>(r))];
        const float2 lq = xc[oc + pad<Fz<K, G>::AB>(roff<K, G, TO>(A - 1 - r))];
        cacc(acc, 1.f, lo, fq);
        l[r] = make_float2(fmaf(-t, lq.y, lo.x), fmaf(t, lq.x, lo.y));
        f[r] = make_float2(fmaf(-t, fq.y, fo.x), fmaf(t, fq.x, fo.y));
        if ((r & 1) == 1) __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// The same with the whole item in one thread's registers (complement partner A-1-r).
template <int A>
__device__ __forceinline__ void reg_flip(float2 (&v)[A], float t) {
#pragma unroll
    for (int r = 0; r < A / 2; ++r) bfly(v[r], v[A - 1 - r], t);
}
template <int A>
__device__ __forceinline__ float reg_unflip2(float2 (&f)[A], float2 (&l)[A], float t) {
    float acc = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) cacc(acc, 1.f, l[r], f[A - 1 - r]);
#pragma unroll
    for (int r = 0; r < A / 2; ++r) {
        bfly(f[r], f[A - 1 - r], -t);
        bfly(l[r], l[A - 1 - r], -t);
    }
    return acc;
}

// Cut values of the thread's amplitudes in stage ST, packed four bytes per register.
template <int K, int G, int ST, int A>
__device__ __forceinline__ void load_cuts(uint32_t (&pk)[(A + 3) / 4], const uint8_t* cut, uint32_t tau) {
    const uint8_t* cb = cut + tbase<K, G, ST>(tau);
#pragma unroll
    for (int w = 0; w < (A + 3) / 4; ++w) pk[w] = 0u;
#pragma unroll
    for (int r = 0; r < A; ++r) pk[r >> 2] |= static_cast<uint32_t>(cb[roff<K, G, ST>(r)]) << (8 * (r & 3));
}

// The packed cut words are loop-invariant; hiding them behind an empty asm at every use
// keeps the compiler from hoisting 2 x A derived addresses into live registers.
template <int A>
__device__ __forceinline__ void opaque(uint32_t (&pk)[(A + 3) / 4]) {
#pragma unroll
    for (int w = 0; w < (A + 3) / 4; ++w) asm volatile("" : "+v"(pk[w]));
}

template <int A>
__device__ __forceinline__ uint32_t cutv(const uint32_t (&pk)[(A + 3) / 4], int r) {
    return (pk[r >> 2] >> (8 * (r & 3))) & 255u;
}

// psi = sc * row[C(x)]: D_1 applied to the uniform state.
template <int A>
__device__ __forceinline__ void gen_stage(float2 (&f)[A], uint32_t (&pk)[(A + 3) / 4], const float2* row,
                                          float sc) {
    opaque<A>(pk);
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 t = row[cutv<A>(pk, r)];
        f[r] = make_float2(sc * t.x, sc * t.y);
        if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
}

template <int A>
__device__ __forceinline__ void phase_stage(float2 (&f)[A], uint32_t (&pk)[(A + 3) / 4], const float2* row,
                                            float sc) {
    opaque<A>(pk);
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 t = row[cutv<A>(pk, r)];
        f[r] = cmul(f[r], make_float2(sc * t.x, sc * t.y));
        if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
}

// Returns the thread's share of Im <lambda| C |psi>; then, with UNDO, applies D^dagger
// scaled by sc (row holds exp(-i gamma c)) to both states.
template <bool UNDO, int A>
__device__ __forceinline__ float cgrad_stage(float2 (&f)[A], float2 (&l)[A], uint32_t (&pk)[(A + 3) / 4],
                                             const float2* row, int cmin, float sc) {
    opaque<A>(pk);
    float a = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const int cq = static_cast<int>(cutv<A>(pk, r));
        cacc(a, static_cast<float>(cq + cmin), l[r], f[r]);
        if constexpr (UNDO) {
            const float2 t0 = row[cq];
            const float2 t = make_float2(sc * t0.x, sc * t0.y);
            f[r] = cmulc(f[r], t);
            l[r] = cmulc(l[r], t);
        }
        if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    return a;
}

// D^dagger scaled by sc on lambda alone, then lambda's share of Im <lambda| C |psi> against
// psi before D (kept from the forward pass): the same term as cgrad_stage takes before its
// undo, since D is diagonal and unimodular.
template <int A>
__device__ __forceinline__ float cterm_lam(float2 (&l)[A], const float2 (&f)[A], uint32_t (&pk)[(A + 3) / 4],
                                           const float2* row, int cmin, float sc) {
    opaque<A>(pk);
    float a = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const int cq = static_cast<int>(cutv<A>(pk, r));
        const float2 t0 = row[cq];
        l[r] = cmulc(l[r], make_float2(sc * t0.x, sc * t0.y));
        cacc(a, static_cast<float>(cq + cmin), l[r], f[r]);
        if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    return a;
}

// Real weights (no common unit, or cut values spanning more than 255 units): the phase of
// every amplitude comes from its own cut value, exp(-i gamma C(x)).  The table holds
// C(x) - c0 (c0 the centre of the cone's cut range: a global phase per layer, which no
// expectation sees, and a smaller argument); the angle gamma (C - c0) / pi is reduced
// modulo 2 in FP64 and its sine and cosine taken in FP32 (sincospif).
__device__ __forceinline__ float2 rphase(double gpi, float c) {
    double x = gpi * static_cast<double>(c);
    x -= 2.0 * rint(0.5 * x);
    float sn, cs;
    sincospif(static_cast<float>(x), &sn, &cs);
    return make_float2(cs, -sn);
}

template <int A>
__device__ __forceinline__ void gen_stage_rw(float2 (&f)[A], const float (&cf)[A], double gpi, float sc) {
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 t = rphase(gpi, cf[r]);
        f[r] = make_float2(sc * t.x, sc * t.y);
    }
}

template <int A>
__device__ __forceinline__ void phase_stage_rw(float2 (&f)[A], const float (&cf)[A], double gpi, float sc) {
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 t = rphase(gpi, cf[r]);
        f[r] = cmul(f[r], make_float2(sc * t.x, sc * t.y));
    }
}

// Im <lambda| C |psi> with C = cf + c0; then, with UNDO, the conjugate phase scaled by sc.
template <bool UNDO, int A>
__device__ __forceinline__ float cgrad_stage_rw(float2 (&f)[A], float2 (&l)[A], const float (&cf)[A], double gpi,
                                                float c0, float sc) {
    float a = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        cacc(a, cf[r] + c0, l[r], f[r]);
        if constexpr (UNDO) {
            const float2 t0 = rphase(gpi, cf[r]);
            const float2 t = make_float2(sc * t0.x, sc * t0.y);
            f[r] = cmulc(f[r], t);
            l[r] = cmulc(l[r], t);
        }
    }
    return a;
}

template <int A>
__device__ __forceinline__ float cterm_lam_rw(float2 (&l)[A], const float2 (&f)[A], const float (&cf)[A], double gpi,
                                              float c0, float sc) {
    float a = 0.f;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 t0 = rphase(gpi, cf[r]);
        l[r] = cmulc(l[r], make_float2(sc * t0.x, sc * t0.y));
        cacc(a, cf[r] + c0, l[r], f[r]);
    }
    return a;
}

template <int K, int G, int ST, int A>
__device__ __forceinline__ void load_cuts_rw(float (&cf)[A], const float* cut, uint32_t tau) {
    const float* cb = cut + tbase<K, G, ST>(tau);
#pragma unroll
    for (int r = 0; r < A; ++r) cf[r] = cb[roff<K, G, ST>(r)];
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// One full mixer layer on a state that sits in the layer's first stage.  Ascending
// layers visit stages 0..S-1, descending ones S-1..0; a layer ends in the stage where
// the next one (of the opposite direction) starts.
// With FLIP the layout holds K stored qubits of a (K+1)-qubit cone and the mixer of the
// dropped qubit rides on the layer's first transpose (or on the registers if there is none).
template <int K, int G, bool DESC, bool FLIP, int A>
__device__ __forceinline__ void fwd_layer(float2 (&f)[A], float2* xb, uint32_t tau, float t) {
    constexpr int S = Fz<K, G>::S;
    static_for<0, S>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr int st = DESC ? S - 1 - j : j;
        if constexpr (j > 0) {
            constexpr int prev = DESC ? S - j : j - 1;
            if constexpr (FLIP && j == 1) xpose_flip<K, G, prev, st>(f, xb, tau, t);
            else xpose<K, G, prev, st>(f, xb, tau);
        }
        mix_stage<K, G, st>(f, t);
    });
    if constexpr (FLIP && S == 1) reg_flip(f, t);
}

// Undo a forward layer of direction DESC on psi and lambda (stages in reverse order);
// returns the thread's share of Im <lambda| sum_j X_j |psi>.
// LAST: the undo of layer 1, whose last stage leaves psi alone (unmix_stage_last).
template <int K, int G, bool DESC, bool FLIP, bool DB, bool LAST = false, int A>
__device__ __forceinline__ double unlayer(float2 (&f)[A], float2 (&l)[A], float2* xb, float2* xb2, uint32_t tau,
                                          float t, float k2) {
    constexpr int S = Fz<K, G>::S;
    double acc = 0.0;
    float w = 1.f;
    if constexpr (FLIP && S == 1) {
        acc += static_cast<double>(w * reg_unflip2(f, l, t));
        w *= k2;
    }
    static_for<0, S>([&](auto J) {
        constexpr int j = decltype(J)::value;            // j-th stage of the reverse walk
        constexpr int st = DESC ? j : S - 1 - j;
        if constexpr (j > 0) {
            constexpr int prev = DESC ? j - 1 : S - j;
            if constexpr (FLIP && j == 1) {
                if constexpr (DB) acc += static_cast<double>(w * xpose2_unflip_dual<K, G, prev, st>(f, l, xb, xb2, tau, t));
                else acc += static_cast<double>(w * xpose2_unflip<K, G, prev, st>(f, l, xb, tau, t));
                w *= k2;
            } else if constexpr (DB) {
                xpose_dual<K, G, prev, st>(f, l, xb, xb2, tau);
            } else {
                xpose<K, G, prev, st>(f, xb, tau);
                xpose<K, G, prev, st>(l, xb, tau);
            }
        }
        if constexpr (LAST && j == S - 1) acc += static_cast<double>(unmix_stage_last<K, G, st>(f, l, t, w));
        else acc += static_cast<double>(unmix_stage2<K, G, st>(f, l, t, k2, w));
    });
    return acc;
}

// ---------------------------------------------------------------- exchange layouts
// Layout variant 3 of the 14-qubit adjoint kernel (13 stored qubits, 16 amplitudes per
// state and thread, 512 threads: lane bits 0-5, wave bits 6-8).  A layout names the qubit
// of every register bit and thread bit.  Four layouts per layer:
//   X0  registers q0-q3,   lanes q4-q9,             waves q10-q12
//   X0s registers q8 q9 q2 q3, lanes q4-q7 q0 q1,   waves q10-q12
//   X1  registers q4-q7,   lanes q12 q0 q1 q2 q10 q11, waves q3 q8 q9
//   X1s registers q10 q11 q6 q7, lanes q12 q0 q1 q2 q4 q5, waves q3 q8 q9
// X0 <-> X0s and X1 <-> X1s exchange register bits 0, 1 with lane bits 4, 5 inside each
// wave (v_permlane16_swap / v_permlane32_swap: no LDS, no barrier); X0s <-> X1 is the one
// LDS transpose of a layer, and the dropped qubit's butterfly rides on it.  A layer mixes
// q0-q3 in X0, q8 q9 in X0s, q4 q5 in X1, and q10 q11 q6 q7 plus q12 (lane bit 0, across
// lanes) in X1s.  X0 holds q0, q1 in register bits 0, 1 like stage 0 of the rotated layouts
// (final mixer, <Z0 Z1>), and X1s stands where their last stage stands.  The lane-bit qubits
// of the transposed layouts (q4-q7 and q12 q0 q1 q2) have padding weights 1, 2, 4, 8 mod 16,
// so each group of 16 lanes hits 16 distinct bank pairs, complement partners included.
struct LayX0 {
    static constexpr int reg[4] = {0, 1, 2, 3};
    static constexpr int thr[9] = {4, 5, 6, 7, 8, 9, 10, 11, 12};
};
struct LayX0s {
    static constexpr int reg[4] = {8, 9, 2, 3};
    static constexpr int thr[9] = {4, 5, 6, 7, 0, 1, 10, 11, 12};
};
struct LayX1 {
    static constexpr int reg[4] = {4, 5, 6, 7};
    static constexpr int thr[9] = {12, 0, 1, 2, 10, 11, 3, 8, 9};
};
struct LayX1s {
    static constexpr int reg[4] = {10, 11, 6, 7};
    static constexpr int thr[9] = {12, 0, 1, 2, 4, 5, 3, 8, 9};
};
template <class L>
__host__ __device__ constexpr uint32_t lay_r(int r) {
    uint32_t q = 0;
    for (int i = 0; i < 4; ++i)
        if ((r >> i) & 1) q |= 1u << L::reg[i];
    return q;
}
template <class L>
__device__ __forceinline__ uint32_t lay_t(uint32_t tau) {
    uint32_t q = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j)
        if ((tau >> j) & 1u) q |= 1u << L::thr[j];
    return q;
}

// Exchange register bits 0, 1 with lane bits 4, 5 (an involution: X0 <-> X0s, X1 <-> X1s).
__device__ __forceinline__ void xswap(float& a, float& b, bool w32) {
    const unsigned x = __float_as_uint(a), y = __float_as_uint(b);
    if (w32) {
        const auto s = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        a = __uint_as_float(s[0]);
        b = __uint_as_float(s[1]);
    } else {
        const auto s = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        a = __uint_as_float(s[0]);
        b = __uint_as_float(s[1]);
    }
}
template <int A>
__device__ __forceinline__ void lane_exchange(float2 (&v)[A]) {
#pragma unroll
    for (int r = 0; r < A; ++r)
        if (!(r & 1)) { xswap(v[r].x, v[r | 1].x, false); xswap(v[r].y, v[r | 1].y, false); }
#pragma unroll
    for (int r = 0; r < A; ++r)
        if (!(r & 2)) { xswap(v[r].x, v[r | 2].x, true); xswap(v[r].y, v[r | 2].y, true); }
}

// Mixer on the register bits in MASK, and (LANE) on lane bit 0 across lanes.
template <int MASK, bool LANE, int A>
__device__ __forceinline__ void xmix(float2 (&v)[A], float t) {
    if constexpr (LANE) {
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 q = lane_x1(v[r]);
            v[r] = make_float2(fmaf(t, q.y, v[r].x), fmaf(-t, q.x, v[r].y));
            if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!((MASK >> i) & 1)) continue;
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

// Undo of xmix on psi and lambda with the terms of Im <lambda| X_j |psi> (as unmix_stage2).
template <int MASK, bool LANE, int A>
__device__ __forceinline__ float xunmix2(float2 (&f)[A], float2 (&l)[A], float t, float k2, float& w) {
    float acc = 0.f;
    if constexpr (LANE) {
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 fq = lane_x1(f[r]);
            const float2 lq = lane_x1(l[r]);
            cacc(a, 1.f, l[r], fq);
            f[r] = make_float2(fmaf(-t, fq.y, f[r].x), fmaf(t, fq.x, f[r].y));
            l[r] = make_float2(fmaf(-t, lq.y, l[r].x), fmaf(t, lq.x, l[r].y));
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        acc = w * a;
        w *= k2;
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!((MASK >> i) & 1)) continue;
        float a0 = 0.f, a1 = 0.f;
        int np = 0;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & (1 << i))) {
                const int r2 = r | (1 << i);
                bfly(f[r], f[r2], -t);
                bfly(l[r], l[r2], -t);
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

// The last step of the undo of layer 1 (as unmix_stage_last): every term at the entry,
// then the mixer undone on lambda alone.
template <int MASK, bool LANE, int A>
__device__ __forceinline__ float xunmix_last(const float2 (&f)[A], float2 (&l)[A], float t, float w) {
    float a0 = 0.f, a1 = 0.f;
    if constexpr (LANE) {
#pragma unroll
        for (int r = 0; r < A; ++r) {
            if (r & 1) cacc(a1, 1.f, l[r], lane_x1(f[r]));
            else cacc(a0, 1.f, l[r], lane_x1(f[r]));
            if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!((MASK >> i) & 1)) continue;
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
    if constexpr (LANE) {
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 lq = lane_x1(l[r]);
            l[r] = make_float2(fmaf(-t, lq.y, l[r].x), fmaf(t, lq.x, l[r].y));
            if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (!((MASK >> i) & 1)) continue;
        int nb = 0;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & (1 << i))) {
                bfly(l[r], l[r | (1 << i)], -t);
                if ((++nb & 7) == 0) __builtin_amdgcn_sched_barrier(0);
            }
        __builtin_amdgcn_sched_barrier(0);
    }
    return w * (a0 + a1);
}

// LDS transpose FROM -> TO with the dropped qubit's butterfly (partner: the complement over
// the stored bits, thread ~tau, register A-1-r), as xpose_flip.
template <class LF, class LT, int A>
__device__ __forceinline__ void xl_flip(float2 (&v)[A], float2* xb, uint32_t tau, float t) {
    constexpr uint32_t TM = 511u;
    float2* pf = xb + opaque_u32(pad<4>(lay_t<LF>(tau)));
    const float2* pt = xb + opaque_u32(pad<4>(lay_t<LT>(tau)));
    const float2* pc = xb + opaque_u32(pad<4>(lay_t<LT>(~tau & TM)));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) pf[pad<4>(lay_r<LF>(r))] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const float2 a = pt[pad<4>(lay_r<LT>(r))];
        const float2 b = pc[pad<4>(lay_r<LT>(A - 1 - r))];
        v[r] = make_float2(fmaf(t, b.y, a.x), fmaf(-t, b.x, a.y));
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
}

// LDS transpose FROM -> TO of psi and lambda undoing the dropped qubit's butterfly; returns
// the thread's share of Im <lambda| X_(K-1) |psi> on the values before the undo (as
// xpose2_unflip_dual / xpose2_unflip).
template <class LF, class LT, bool DB, int A>
__device__ __forceinline__ float xl_unflip2(float2 (&f)[A], float2 (&l)[A], float2* xa, float2* xc, uint32_t tau,
                                            float t) {
    constexpr uint32_t TM = 511u;
    const uint32_t of = opaque_u32(pad<4>(lay_t<LF>(tau)));
    const uint32_t ot = opaque_u32(pad<4>(lay_t<LT>(tau)));
    const uint32_t oc = opaque_u32(pad<4>(lay_t<LT>(~tau & TM)));
    float acc = 0.f;
    if constexpr (DB) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < A; ++r) {
            xa[of + pad<4>(lay_r<LF>(r))] = f[r];
            xc[of + pad<4>(lay_r<LF>(r))] = l[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 fo = xa[ot + pad<4>(lay_r<LT>(r))];
            const float2 fq = xa[oc + pad<4>(lay_r<LT>(A - 1 - r))];
            const float2 lo = xc[ot + pad<4>(lay_r<LT>(r))];
            const float2 lq = xc[oc + pad<4>(lay_r<LT>(A - 1 - r))];
            cacc(acc, 1.f, lo, fq);
            l[r] = make_float2(fmaf(-t, lq.y, lo.x), fmaf(t, lq.x, lo.y));
            f[r] = make_float2(fmaf(-t, fq.y, fo.x), fmaf(t, fq.x, fo.y));
            if ((r & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        float2 fp[A];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < A; ++r) xa[of + pad<4>(lay_r<LF>(r))] = f[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < A; ++r) {
            f[r] = xa[ot + pad<4>(lay_r<LT>(r))];
            fp[r] = xa[oc + pad<4>(lay_r<LT>(A - 1 - r))];
            if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < A; ++r) xa[of + pad<4>(lay_r<LF>(r))] = l[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < A; ++r) {
            const float2 lo = xa[ot + pad<4>(lay_r<LT>(r))];
            const float2 lq = xa[oc + pad<4>(lay_r<LT>(A - 1 - r))];
            cacc(acc, 1.f, lo, fp[r]);
            l[r] = make_float2(fmaf(-t, lq.y, lo.x), fmaf(t, lq.x, lo.y));
            f[r] = make_float2(fmaf(-t, fp[r].y, f[r].x), fmaf(t, fp[r].x, f[r].y));
            if ((r & 1) == 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
    return acc;
}

// One forward layer in the exchange layouts: descending X1s -> X1 -> X0s -> X0, ascending
// the reverse; the dropped qubit on the transpose.
template <bool DESC, int A>
__device__ __forceinline__ void xfwd_layer(float2 (&f)[A], float2* xb, uint32_t tau, float t) {
    static_assert(A == 16, "exchange layouts hold 16 amplitudes per thread");
    if constexpr (DESC) {
        xmix<0xF, true>(f, t);
        lane_exchange(f);
        xmix<0x3, false>(f, t);
        xl_flip<LayX1, LayX0s>(f, xb, tau, t);
        xmix<0x3, false>(f, t);
        lane_exchange(f);
        xmix<0xF, false>(f, t);
    } else {
        xmix<0xF, false>(f, t);
        lane_exchange(f);
        xmix<0x3, false>(f, t);
        xl_flip<LayX0s, LayX1>(f, xb, tau, t);
        xmix<0x3, false>(f, t);
        lane_exchange(f);
        xmix<0xF, true>(f, t);
    }
}

// Undo a forward layer of direction DESC on psi and lambda; returns the thread's share of
// Im <lambda| sum_j X_j |psi>.  LAST: the undo of layer 1 (xunmix_last in its last layout).
template <bool DESC, bool DB, bool LAST, int A>
__device__ __forceinline__ double xunlayer(float2 (&f)[A], float2 (&l)[A], float2* xb, float2* xb2, uint32_t tau,
                                           float t, float k2) {
    static_assert(A == 16, "exchange layouts hold 16 amplitudes per thread");
    double acc = 0.0;
    float w = 1.f;
    if constexpr (DESC) {   // X0 -> X0s -> X1 -> X1s
        acc += static_cast<double>(xunmix2<0xF, false>(f, l, t, k2, w));
        lane_exchange(f);
        lane_exchange(l);
        acc += static_cast<double>(xunmix2<0x3, false>(f, l, t, k2, w));
        acc += static_cast<double>(w * xl_unflip2<LayX0s, LayX1, DB>(f, l, xb, DB ? xb2 : xb, tau, t));
        w *= k2;
        acc += static_cast<double>(xunmix2<0x3, false>(f, l, t, k2, w));
        lane_exchange(f);
        lane_exchange(l);
        if constexpr (LAST) acc += static_cast<double>(xunmix_last<0xF, true>(f, l, t, w));
        else acc += static_cast<double>(xunmix2<0xF, true>(f, l, t, k2, w));
    } else {                // X1s -> X1 -> X0s -> X0
        acc += static_cast<double>(xunmix2<0xF, true>(f, l, t, k2, w));
        lane_exchange(f);
        lane_exchange(l);
        acc += static_cast<double>(xunmix2<0x3, false>(f, l, t, k2, w));
        acc += static_cast<double>(w * xl_unflip2<LayX1, LayX0s, DB>(f, l, xb, DB ? xb2 : xb, tau, t));
        w *= k2;
        acc += static_cast<double>(xunmix2<0x3, false>(f, l, t, k2, w));
        lane_exchange(f);
        lane_exchange(l);
        if constexpr (LAST) acc += static_cast<double>(xunmix_last<0xF, false>(f, l, t, w));
        else acc += static_cast<double>(xunmix2<0xF, false>(f, l, t, k2, w));
    }
    return acc;
}

// Cut values of the thread's amplitudes in layout L, packed four bytes per register, or
// floats (real weights).
template <class L, int A>
__device__ __forceinline__ void xload_cuts(uint32_t (&pk)[(A + 3) / 4], const uint8_t* cut, uint32_t tau) {
    const uint8_t* cb = cut + lay_t<L>(tau);
#pragma unroll
    for (int w = 0; w < (A + 3) / 4; ++w) pk[w] = 0u;
#pragma unroll
    for (int r = 0; r < A; ++r) pk[r >> 2] |= static_cast<uint32_t>(cb[lay_r<L>(r)]) << (8 * (r & 3));
}
template <class L, int A>
__device__ __forceinline__ void xload_cuts_rw(float (&cf)[A], const float* cut, uint32_t tau) {
    const float* cb = cut + lay_t<L>(tau);
#pragma unroll
    for (int r = 0; r < A; ++r) cf[r] = cb[lay_r<L>(r)];
}

// Sum over the threads of one item (fixed order, identical result in every lane).
template <int K, int G>
__device__ __forceinline__ double item_sum(double x, double* red, int tid) {
    using C = Fz<K, G>;
    constexpr int seg = C::TPI < 64 ? C::TPI : 64;
#pragma unroll
    for (int o = 1; o < seg; o <<= 1) x += __shfl_xor(x, o, 64);
    if constexpr (C::TPI > 64) {
        constexpr int WPI = C::TPI / 64;
        const int wave = tid >> 6;
        __syncthreads();
        if ((tid & 63) == 0) red[wave] = x;
        __syncthreads();
        const int w0 = (wave / WPI) * WPI;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WPI; ++w) s += red[w0 + w];
        x = s;
    }
    return x;
}

// ODD = (p - 1) is odd.  Layer l (1 <= l <= p-1) runs descending when p-1-l is even, so
// layer p-1 ends in stage 0 (qubits 0 and 1).  With ODD the first layer is descending and
// is peeled off; the remaining layers come in (ascending, descending) pairs, so no branch
// ever selects between the two layer bodies.
// RW: real weights (cut_tables then holds float C(x) - c0 per cone; no phase rows).
template <int K, bool GRAD, bool ODD, bool DB, bool GR, bool RW = false, int V = 0>
__global__ void __launch_bounds__((Fz<(K >= 3 ? K - 1 : K), (GRAD ? 1 : 0) | (V << 1)>::WG))
k_fused(const ConeDev* __restrict__ cones, int64_t item_base, int64_t n_items,
        const uint8_t* __restrict__ cut_tables, int32_t rowcap, EvalArgs ea) {
    constexpr int GI = (GRAD ? 1 : 0) | (V << 1);
    // FLIP: the state is stored on KL = K - 1 qubits (global-flip halving); every sum over
    // the stored half is half the sum over the whole state
    constexpr bool FLIP = K >= 3;
    constexpr int KL = FLIP ? K - 1 : K;
    constexpr double HS = FLIP ? 2.0 : 1.0;
    using C = Fz<KL, GI>;
    constexpr int A = C::A;
    // variant 3: the exchange layouts (14-qubit adjoint only)
    constexpr bool XL = V == 3;
    static_assert(!XL || (KL == 13 && GRAD && A == 16 && C::TPI == 512), "exchange layouts: 14-qubit adjoint only");
    __shared__ float2 xbuf[C::S > 1 ? (DB ? 2 : 1) * C::IPW * C::NPAD : 1];
    // cut table of each item: bytes (C - cut_min) or, with RW, floats (C - c0)
    constexpr int CUTB = (RW ? 4 : 1) * C::IPW * C::N;
    __shared__ __attribute__((aligned(16))) uint8_t cutl[CUTB < 16 ? 16 : CUTB];
    __shared__ double red[C::WG / 64];
    // Deferred item sums (items of more than one wave): every value is summed within its
    // wave at once (no barrier); the per-wave partials wait in LDS with the code of their
    // destination and are summed over the item's waves and written at a flush, in the
    // order item_sum uses, so one barrier pair serves up to NSUM values.
    constexpr bool DEFER = C::TPI > 64;
    constexpr int NSUM = 8;
    __shared__ double dsum[DEFER ? NSUM : 1][DEFER ? C::WG / 64 : 1];
    __shared__ int32_t dcode[DEFER ? NSUM : 1];
    int nsum = 0;
    extern __shared__ float2 prow_all[];   // [IPW][p][rowcap] phase rows of every layer

    const int tid = threadIdx.x;
    const int il = tid >> C::TB;
    const uint32_t tau = static_cast<uint32_t>(tid) & (C::TPI - 1);
    int64_t item = item_base + static_cast<int64_t>(blockIdx.x) * C::IPW + il;
    const bool valid = item < n_items;
    if (!valid) item = n_items - 1;
    const int P = ea.P, p = ea.p;
    const int64_t slot = item / P;
    const int point = static_cast<int>(item - slot * P);
    const ConeDev cd = cones[slot];

    if constexpr (RW) {   // the cone's float cut table -> LDS (each thread copies A floats)
        const float* src = reinterpret_cast<const float*>(cut_tables) + cd.cut_off + static_cast<size_t>(tau) * A;
        float* dst = reinterpret_cast<float*>(cutl) + il * C::N + tau * A;
#pragma unroll
        for (int j = 0; j < A; ++j) dst[j] = src[j];
    } else {   // the cone's cut table -> LDS (each thread copies A bytes)
        const uint8_t* src = cut_tables + cd.cut_off + static_cast<size_t>(tau) * A;
        uint8_t* dst = cutl + il * C::N + tau * A;
        if constexpr (A >= 16) {
#pragma unroll
            for (int j = 0; j < A; j += 16)
                *reinterpret_cast<uint4*>(dst + j) = *reinterpret_cast<const uint4*>(src + j);
        } else {
#pragma unroll
            for (int j = 0; j < A; ++j) dst[j] = src[j];
        }
    }
    const uint8_t* cut = cutl + il * C::N;
    const float* cutf = reinterpret_cast<const float*>(cutl) + il * C::N;
    float2* xb = xbuf + (C::S > 1 ? il * C::NPAD : 0);
    float2* xb2 = DB ? xbuf + (C::S > 1 ? (C::IPW + il) * C::NPAD : 0) : nullptr;
    const size_t ipt = static_cast<size_t>(cd.inst) * P + point;   // angle point of the cone's instance
    const float2* phase0 = ea.phase + ipt * p * ea.R + cd.cut_shift;
    const float2* mix0 = ea.mix + ipt * p;
    // phase rows of every layer for this item: prow[il][l][c] = exp(-i gamma_l (cut_min + c)),
    // staged in LDS; GR: they do not fit beside the kernel's LDS (deep circuits with many
    // items per workgroup) and are read from the table in device memory instead
    if constexpr (!GR && !RW) {
        float2* dst = prow_all + static_cast<size_t>(il) * p * rowcap;
        for (int l = 0; l < p; ++l)
            for (int c = static_cast<int>(tau); c < cd.cut_range; c += C::TPI)
                dst[l * rowcap + c] = phase0[static_cast<size_t>(l) * ea.R + c];
    }
    const float2* rows = GR ? phase0 : prow_all + static_cast<size_t>(il) * p * rowcap;
    const int rstride = GR ? ea.R : rowcap;
    auto ROW = [&](int l) { return rows + l * rstride; };
    constexpr int SL = C::S - 1;
    constexpr int NW = (A + 3) / 4;
    __syncthreads();
    // cut values of the thread's amplitudes in stages 0 and SL: packed bytes, or floats (RW)
    uint32_t pk0[RW ? 1 : NW], pkL[RW ? 1 : NW];
    float cf0[RW ? A : 1], cfL[RW ? A : 1];
    if constexpr (RW) {
        if constexpr (XL) {
            xload_cuts_rw<LayX0, A>(cf0, cutf, tau);
            xload_cuts_rw<LayX1s, A>(cfL, cutf, tau);
        } else {
            load_cuts_rw<KL, GI, 0, A>(cf0, cutf, tau);
            load_cuts_rw<KL, GI, SL, A>(cfL, cutf, tau);
        }
    } else if constexpr (XL) {
        xload_cuts<LayX0, A>(pk0, cut, tau);
        xload_cuts<LayX1s, A>(pkL, cut, tau);
    } else {
        load_cuts<KL, GI, 0, A>(pk0, cut, tau);
        load_cuts<KL, GI, SL, A>(pkL, cut, tau);
    }
    // gamma_l / pi of this item's point (real weights)
    const double* gam = RW ? ea.gamma + (static_cast<size_t>(cd.inst) * ea.gamma_P + point) * p : nullptr;
    auto GPI = [&](int l) { return gam[l] * 0.31830988618379067154; };
    // mix0[l] = (tau_l, |kappa_l|^2); a full factored layer scales the state by
    // 1/|kappa|^K, the truncated last layer (qubits 0, 1) by 1/|kappa_p|^2.
    auto kpowK = [&](float k2) { return exp2f(0.5f * K * log2f(k2)); };
    const float k2p = mix0[p - 1].y;
    // code 0: <Z0 Z1> of the item; code 1 + j: entry j of its gradient (gamma_1..p, beta_1..p)
    auto put_out = [&](int code, double x) {
        if (!valid) return;
        if (code == 0) ea.zz[static_cast<size_t>(point) * ea.M + cd.orbit] = x;
        else ea.g[(static_cast<size_t>(point) * 2 * p + (code - 1)) * ea.M + cd.orbit] = x;
    };
    auto flush = [&]() {
        if constexpr (DEFER) {
            __syncthreads();
            if (tau == 0) {
                const int w0 = tid >> 6;   // the item's first wave
                for (int q = 0; q < nsum; ++q) {
                    double x = 0.0;
#pragma unroll
                    for (int w = 0; w < C::TPI / 64; ++w) x += dsum[q][w0 + w];
                    put_out(dcode[q], x);
                }
            }
            __syncthreads();
            nsum = 0;
        }
    };
    auto put = [&](int code, double x) {
        if constexpr (DEFER) {
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
            if ((tid & 63) == 0) dsum[nsum][tid >> 6] = x;
            if (tid == 0) dcode[nsum] = code;
            if (++nsum == NSUM) flush();
        } else {
            x = item_sum<KL, GI>(x, red, tid);
            if (tau == 0) put_out(code, x);
        }
    };

    float2 f[A];
    // GRAD: psi after the mixer of layer p-1 at its true norm, kept for the adjoint (which
    // then undoes D_p and the last mixer on lambda alone)
    float2 f1[GRAD ? A : 1];
    // ---- D_1 |+>, then the full layers 1..p-1, each followed by the next phase.
    // Phase row l (0-based) is scaled by the norm lost in the layer before it, and the
    // last one also by |kappa_p|^2, so psi leaves the final mixer normalised.
    {
        const float sc = exp2f(-0.5f * K) * (p == 1 ? k2p : 1.f);
        if constexpr (RW) gen_stage_rw(f, ODD ? cfL : cf0, GPI(0), sc);
        else if constexpr (ODD) gen_stage(f, pkL, ROW(0), sc);
        else gen_stage(f, pk0, ROW(0), sc);
    }
    // the phase after a descending layer l (stage 0); kk = |kappa_l|^K
    auto phase_desc = [&](int l, float kk) {
        if (GRAD && l + 1 == p) {
#pragma unroll
            for (int r = 0; r < A; ++r) {
                f[r] = make_float2(kk * f[r].x, kk * f[r].y);
                if constexpr (GRAD) f1[r] = f[r];
            }
            kk = 1.f;
        }
        const float sc = kk * (l + 1 == p ? k2p : 1.f);
        if constexpr (RW) phase_stage_rw(f, cf0, GPI(l), sc);
        else phase_stage(f, pk0, ROW(l), sc);
    };
    int l1 = 1;
    if constexpr (ODD) {
        const float2 tk = mix0[0];
        if constexpr (XL) xfwd_layer<true>(f, xb, tau, tk.x);
        else fwd_layer<KL, GI, true, FLIP>(f, xb, tau, tk.x);
        phase_desc(1, kpowK(tk.y));
        l1 = 2;
    }
    for (; l1 + 1 <= p - 1; l1 += 2) {
        const float2 ta = mix0[l1 - 1];
        if constexpr (XL) xfwd_layer<false>(f, xb, tau, ta.x);
        else fwd_layer<KL, GI, false, FLIP>(f, xb, tau, ta.x);
        if constexpr (RW) phase_stage_rw(f, cfL, GPI(l1), kpowK(ta.y));
        else phase_stage(f, pkL, ROW(l1), kpowK(ta.y));
        const float2 tb = mix0[l1];
        if constexpr (XL) xfwd_layer<true>(f, xb, tau, tb.x);
        else fwd_layer<KL, GI, true, FLIP>(f, xb, tau, tb.x);
        phase_desc(l1 + 1, kpowK(tb.y));
    }

    // ---- last layer: mixer on qubits 0, 1 (register bits 0, 1 of stage 0); <Z0 Z1>
    const float tp = mix0[p - 1].x;
#pragma unroll
    for (int r = 0; r < A; ++r)
        if (!(r & 1)) bfly(f[r], f[r | 1], tp);
#pragma unroll
    for (int r = 0; r < A; ++r)
        if (!(r & 2)) bfly(f[r], f[r | 2], tp);
    double zzp = 0.0;
#pragma unroll
    for (int r = 0; r < A; ++r) {
        const double pr = static_cast<double>(fmaf(f[r].x, f[r].x, f[r].y * f[r].y));
        zzp += (((r ^ (r >> 1)) & 1) ? -pr : pr);
    }
    put(0, HS * zzp);

    if constexpr (GRAD) {
        float2 lam[A];
#pragma unroll
        for (int r = 0; r < A; ++r) lam[r] = (((r ^ (r >> 1)) & 1) ? make_float2(-f[r].x, -f[r].y) : f[r]);
        // d zz / d beta_p: only X_0, X_1 contribute in the truncated last layer
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & 1)) xacc(acc, lam[r], lam[r | 1], f[r], f[r | 1]);
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & 2)) xacc(acc, lam[r], lam[r | 2], f[r], f[r | 2]);
        put(2 * p, HS * 2.0 * static_cast<double>(acc));
        const float mup = k2p;   // the undone last mixer leaves lambda scaled by 1/|kappa_p|^2
        if (p == 1) {
            // undo the last mixer on both states; the gamma_1 term (both carry 1/mu_p)
#pragma unroll
            for (int r = 0; r < A; ++r)
                if (!(r & 2)) { bfly(f[r], f[r | 2], -tp); bfly(lam[r], lam[r | 2], -tp); }
#pragma unroll
            for (int r = 0; r < A; ++r)
                if (!(r & 1)) { bfly(f[r], f[r | 1], -tp); bfly(lam[r], lam[r | 1], -tp); }
            float a;
            if constexpr (RW) a = cgrad_stage_rw<false>(f, lam, cf0, 0.0, cd.c0, 1.f);
            else a = cgrad_stage<false>(f, lam, pk0, ROW(0), cd.cut_min, 1.f);
            put(1, HS * 2.0 * static_cast<double>(mup) * mup * a);
            flush();
            return;
        }
        // undo the last mixer on lambda; then D_p on lambda (the row scaled by mu_p restores
        // its true norm) with the gamma_p term against the kept psi
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & 2)) bfly(lam[r], lam[r | 2], -tp);
#pragma unroll
        for (int r = 0; r < A; ++r)
            if (!(r & 1)) bfly(lam[r], lam[r | 1], -tp);
        {
            float a;
            if constexpr (RW) a = cterm_lam_rw(lam, f1, cf0, GPI(p - 1), cd.c0, mup);
            else a = cterm_lam(lam, f1, pk0, ROW(p - 1), cd.cut_min, mup);
            put(p, HS * 2.0 * static_cast<double>(a));
        }
#pragma unroll
        for (int r = 0; r < A; ++r) f[r] = f1[r];

        // The undo of layer 1 (descending iff ODD) leaves psi alone in its last stage and
        // regenerates D_1 |+> in the stage it ends in for the gamma_1 term (lambda carries
        // 1/mu_1, mu_1 = |kappa_1|^K; psi is exact).
        auto last_layer = [&](auto dir) {
            constexpr bool D = decltype(dir)::value;
            const float2 tk = mix0[0];
            double b;
            if constexpr (XL) b = xunlayer<D, DB, true>(f, lam, xb, xb2, tau, tk.x, tk.y);
            else b = unlayer<KL, GI, D, FLIP, DB, true>(f, lam, xb, xb2, tau, tk.x, tk.y);
            put(1 + p, HS * 2.0 * b);
            const float mu = kpowK(tk.y);
            const float sc = exp2f(-0.5f * K);
            float a;
            if constexpr (RW) {
                gen_stage_rw(f, D ? cfL : cf0, GPI(0), sc);
                a = cgrad_stage_rw<false>(f, lam, D ? cfL : cf0, 0.0, cd.c0, 1.f);
            } else if constexpr (D) {
                gen_stage(f, pkL, ROW(0), sc);
                a = cgrad_stage<false>(f, lam, pkL, ROW(0), cd.cut_min, 1.f);
            } else {
                gen_stage(f, pk0, ROW(0), sc);
                a = cgrad_stage<false>(f, lam, pk0, ROW(0), cd.cut_min, 1.f);
            }
            put(1, HS * 2.0 * static_cast<double>(mu) * a);
        };

        // Walk layers p-1 .. 2 back (both states exact at the start of each).  Layer p-1 is
        // descending (stage 0 -> SL); the layers then alternate.  Undoing layer l leaves both
        // states scaled by 1/mu_l (mu_l = |kappa_l|^K); D_l is then undone with a row scaled
        // by mu_l, which restores them.
        int ly = p;
        for (;;) {
            if (ly == 2) {
                if constexpr (ODD) last_layer(std::true_type{});
                break;
            }
            float mu;
            {
                const float2 tk = mix0[ly - 2];
                double b;
                if constexpr (XL) b = xunlayer<true, DB, false>(f, lam, xb, xb2, tau, tk.x, tk.y);
                else b = unlayer<KL, GI, true, FLIP, DB>(f, lam, xb, xb2, tau, tk.x, tk.y);
                put(1 + p + ly - 2, HS * 2.0 * b);
                mu = kpowK(tk.y);
            }
            --ly;
            {
                float a;
                if constexpr (RW) a = cgrad_stage_rw<true>(f, lam, cfL, GPI(ly - 1), cd.c0, mu);
                else a = cgrad_stage<true>(f, lam, pkL, ROW(ly - 1), cd.cut_min, mu);
                put(ly, HS * 2.0 * static_cast<double>(mu) * mu * a);
            }
            if (ly == 2) {
                if constexpr (!ODD) last_layer(std::false_type{});
                break;
            }
            {
                const float2 tk = mix0[ly - 2];
                double b;
                if constexpr (XL) b = xunlayer<false, DB, false>(f, lam, xb, xb2, tau, tk.x, tk.y);
                else b = unlayer<KL, GI, false, FLIP, DB>(f, lam, xb, xb2, tau, tk.x, tk.y);
                put(1 + p + ly - 2, HS * 2.0 * b);
                mu = kpowK(tk.y);
            }
            --ly;
            {
                float a;
                if constexpr (RW) a = cgrad_stage_rw<true>(f, lam, cf0, GPI(ly - 1), cd.c0, mu);
                else a = cgrad_stage<true>(f, lam, pk0, ROW(ly - 1), cd.cut_min, mu);
                put(ly, HS * 2.0 * static_cast<double>(mu) * mu * a);
            }
        }
    }
    flush();
}

// ---------------------------------------------------------------- launcher
// LDS bytes a kernel variant declares statically (queried once per variant; concurrent
// first calls may both query, which is harmless)
template <int K, bool GRAD, bool ODD, bool DB, bool GR, int V>
hipError_t static_lds(size_t& out) {
    static std::atomic<size_t> bytes{0};   // + 1 once queried
    size_t b = bytes.load(std::memory_order_relaxed);
    if (!b) {
        hipFuncAttributes fa{};
        const hipError_t e =
            hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_fused<K, GRAD, ODD, DB, GR, false, V>));
        if (e != hipSuccess) return e;
        b = fa.sharedSizeBytes + 1;
        bytes.store(b, std::memory_order_relaxed);
    }
    out = b - 1;
    return hipSuccess;
}

// Picks the kernel whose LDS holds the phase rows (dyn bytes): two transpose buffers
// (adjoint, 13 and 14 qubits) when they fit, else one, else rows stay in device memory;
// real weights need no rows.
template <int K, bool GRAD, bool ODD, int V>
hipError_t launch_v(dim3 grid, dim3 block, size_t dyn, const ConeDev* cones, int64_t item_base, int64_t n_items,
                    const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    constexpr size_t LDS_MAX = 160 * 1024;
    size_t lds = 0;
    hipError_t e;
    if (ea.realw) {   // real weights: phases per amplitude, no rows in LDS
        hipLaunchKernelGGL((k_fused<K, GRAD, ODD, false, false, true, V>), grid, block, 0, st, cones, item_base,
                           n_items, cut, 0, ea);
        return hipGetLastError();
    }
    if constexpr (GRAD && K >= 13) {
        if ((e = static_lds<K, GRAD, ODD, true, false, V>(lds)) != hipSuccess) return e;
        if (lds + dyn <= LDS_MAX) {
            hipLaunchKernelGGL((k_fused<K, GRAD, ODD, true, false, false, V>), grid, block, dyn, st, cones, item_base,
                               n_items, cut, rowcap, ea);
            return hipGetLastError();
        }
    }
    if ((e = static_lds<K, GRAD, ODD, false, false, V>(lds)) != hipSuccess) return e;
    if (lds + dyn <= LDS_MAX)
        hipLaunchKernelGGL((k_fused<K, GRAD, ODD, false, false, false, V>), grid, block, dyn, st, cones, item_base,
                           n_items, cut, rowcap, ea);
    else
        hipLaunchKernelGGL((k_fused<K, GRAD, ODD, false, true, false, V>), grid, block, 0, st, cones, item_base,
                           n_items, cut, -1, ea);
    return hipGetLastError();
}

// Variants of the K-qubit kernel that differ from the default layout (Fz): 1 needs more
// stored qubits than the default register bits minus one, 2 fewer threads per item than 256,
// 3 (the exchange layouts) is the 14-qubit adjoint kernel only.
template <int K>
constexpr bool fused_variant_ok(bool grad, int v) {
    constexpr int KL = K >= 3 ? K - 1 : K;
    if (v == 0) return true;
    if (v == 1) return grad ? KL >= QAOA_FUSED_AB_GRAD : KL >= 5;
    if (v == 3) return grad && K == 14 && QAOA_FUSED_AB_GRAD == 4;
    return grad ? Fz<KL, 1>::TPI < 256 : Fz<KL, 0>::TPI < 256;
}

template <int K, int V>
hipError_t launch_kv(bool grad, const ConeDev* cones, int64_t item_base, int64_t n_items, const uint8_t* cut,
                     int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    constexpr int KL = K >= 3 ? K - 1 : K;   // stored qubits (global-flip halving)
    const int ipw = grad ? Fz<KL, 1 | (V << 1)>::IPW : Fz<KL, V << 1>::IPW;
    const int wg = grad ? Fz<KL, 1 | (V << 1)>::WG : Fz<KL, V << 1>::WG;
    const int64_t todo = n_items - item_base;
    const int64_t blocks = (todo + ipw - 1) / ipw;
    if (blocks <= 0) return hipSuccess;
    const size_t dyn = static_cast<size_t>(ipw) * ea.p * rowcap * sizeof(float2);
    const dim3 block(wg);
    const bool odd = ((ea.p - 1) & 1) != 0;
    // a grid holds fewer than 2^32 threads (work-items): larger batches take several launches
    const int64_t max_blocks = static_cast<int64_t>(UINT32_MAX) / wg;
    for (int64_t b0 = 0; b0 < blocks; b0 += max_blocks) {
        const dim3 grid(static_cast<unsigned>(std::min(max_blocks, blocks - b0)));
        const int64_t base = item_base + b0 * ipw;
        hipError_t e;
        if (grad) {
            e = odd ? launch_v<K, true, true, V>(grid, block, dyn, cones, base, n_items, cut, rowcap, ea, st)
                    : launch_v<K, true, false, V>(grid, block, dyn, cones, base, n_items, cut, rowcap, ea, st);
        } else if constexpr (V != 3) {
            e = odd ? launch_v<K, false, true, V>(grid, block, dyn, cones, base, n_items, cut, rowcap, ea, st)
                    : launch_v<K, false, false, V>(grid, block, dyn, cones, base, n_items, cut, rowcap, ea, st);
        } else {
            return hipErrorInvalidValue;   // the exchange layouts exist for the adjoint only
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// variant: 0, 1, 2, 3 (see Fz and fused_variant_ok); a variant that does not apply to K runs
// the default
template <int K>
hipError_t launch_k(bool grad, int variant, const ConeDev* cones, int64_t item_base, int64_t n_items,
                    const uint8_t* cut, int32_t rowcap, const EvalArgs& ea, hipStream_t st) {
    if (variant == 1 && fused_variant_ok<K>(grad, 1)) {
        if constexpr ((K >= 3 ? K - 1 : K) >= QAOA_FUSED_AB_GRAD)
            return launch_kv<K, 1>(grad, cones, item_base, n_items, cut, rowcap, ea, st);
    }
    if (variant == 2 && fused_variant_ok<K>(grad, 2)) {
        if constexpr (Fz<(K >= 3 ? K - 1 : K), 0>::TPI < 256)
            return launch_kv<K, 2>(grad, cones, item_base, n_items, cut, rowcap, ea, st);
    }
    if (variant == 3 && fused_variant_ok<K>(grad, 3)) {
        if constexpr (K == 14 && QAOA_FUSED_AB_GRAD == 4)
            return launch_kv<K, 3>(grad, cones, item_base, n_items, cut, rowcap, ea, st);
    }
    return launch_kv<K, 0>(grad, cones, item_base, n_items, cut, rowcap, ea, st);
}

}  // namespace qaoa

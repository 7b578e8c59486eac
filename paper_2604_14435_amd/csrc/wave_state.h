// Register-resident state vectors: one wavefront holds 2^(NQ+1) amplitudes,
// 64 lanes x 2^(NQ-5) registers.  Lane bit 5 selects one of two halves (the
// ancilla of a Hadamard-test circuit, or one of two vectors evolved by the
// same gates); the NQ system qubits are split between registers and lane
// bits 0..4 in one of two layouts:
//   LO: register bits = qubits 0..NQ-6, lane bits 0..4 = qubits NQ-5..NQ-1;
//   HI: register bits = qubits 5..NQ-1, lane bits 0..4 = qubits 0..4.
// Gates act on register qubits only; a layout swap goes through LDS.
//
// RY(t) rotates each amplitude pair by phi = t/2, applied as three shears
// a -= tan(phi/2) b; b += sin(phi) a; a -= tan(phi/2) b (six FMAs per complex
// pair) with phi reduced to [-pi/2, pi/2] (the reduction multiplies the
// whole half by -1).
//
// CZ ladder.  The ladder is S = diag((-1)^{Q(g)}), Q(g) = sum_q g_q g_{q+1}.
// The stored amplitudes are S^p times the true ones (p = ladders applied so
// far, mod 2).  S RY_q S rotates by (-1)^{g_{q-1} xor g_{q+1}} t on each pair,
// so with p = 1 every pair uses +-angle: a per-lane sign times a
// compile-time per-register sign.
#pragma once

#include "circuits.h"

namespace dvq {

template <int NQ, bool HI>
struct Lay {
    static constexpr int RB = NQ - 5;
    static constexpr int R = 1 << RB;
    // register bit holding qubit q, or -1
    static constexpr int reg(int q) {
        return HI ? ((q >= 5 && q < NQ) ? q - 5 : -1) : ((q >= 0 && q < RB) ? q : -1);
    }
    // lane bit holding system qubit q, or -1
    static constexpr int lanebit(int q) {
        return HI ? ((q >= 0 && q < 5) ? q : -1) : ((q >= RB && q < NQ) ? q - RB : -1);
    }
    // global basis index of (lane, r); bit NQ is the half
    __device__ static __forceinline__ int g(int lane, int r) {
        return HI ? ((lane & 31) | (r << 5) | ((lane >> 5) << NQ))
                  : (r | ((lane & 31) << RB) | ((lane >> 5) << NQ));
    }
};

// LDS slot of basis index g: one pad amplitude every 32.
__device__ __forceinline__ int pad_slot(int g) { return g + (g >> 5); }

// Sign of the pair (r0, r0 | bit of Q) under the lazy ladder frame: the lane
// part is returned by lane_rho, the register part by reg_rho.
template <int NQ, bool HI, int Q>
__device__ __forceinline__ int lane_rho(int lane) {
    using Ly = Lay<NQ, HI>;
    constexpr int lm = Q > 0 ? Ly::lanebit(Q - 1) : -1;
    constexpr int lp = Q + 1 < NQ ? Ly::lanebit(Q + 1) : -1;
    int rl = 0;
    if constexpr (lm >= 0) rl ^= lane >> lm;
    if constexpr (lp >= 0) rl ^= lane >> lp;
    return rl & 1;
}

template <int NQ, bool HI, int Q>
__host__ __device__ constexpr bool reg_rho(int r0) {
    using Ly = Lay<NQ, HI>;
    constexpr int rm = Q > 0 ? Ly::reg(Q - 1) : -1;
    constexpr int rp = Q + 1 < NQ ? Ly::reg(Q + 1) : -1;
    bool neg = false;
    if (rm >= 0) neg ^= (r0 >> rm) & 1;
    if (rp >= 0) neg ^= (r0 >> rp) & 1;
    return neg;
}

template <typename T, int NQ, bool HI, int Q, int PAR>
__device__ __forceinline__ void ry_reg(T* re, T* im, int lane, T t, T s) {
    using Ly = Lay<NQ, HI>;
    constexpr int R = Ly::R;
    constexpr int j = Ly::reg(Q);
    static_assert(j >= 0, "qubit not in registers");
    T tp = t, sp = s;
    if constexpr (PAR) {
        if (lane_rho<NQ, HI, Q>(lane)) {
            tp = -t;
            sp = -s;
        }
    }
    const T mtp = -tp, mtn = tp, spp = sp, spn = -sp;
#pragma unroll
    for (int r0 = 0; r0 < R; ++r0) {
        if (r0 & (1 << j)) continue;
        const int r1 = r0 | (1 << j);
        const bool neg = PAR ? reg_rho<NQ, HI, Q>(r0) : false;
        const T mt = neg ? mtn : mtp;
        const T ss = neg ? spn : spp;
        re[r0] = fmat(mt, re[r1], re[r0]);
        im[r0] = fmat(mt, im[r1], im[r0]);
        re[r1] = fmat(ss, re[r0], re[r1]);
        im[r1] = fmat(ss, im[r0], im[r1]);
        re[r0] = fmat(mt, re[r1], re[r0]);
        im[r0] = fmat(mt, im[r1], im[r0]);
    }
}

// RY on every qubit q in [Q, QEND) that is a register qubit of the layout;
// trig[2k], trig[2k+1] = tan(phi_k/2), sin(phi_k); `sign` = +1 applies the
// gates, -1 their inverses.
template <typename T, int NQ, bool HI, int PAR, int Q, int QEND>
__device__ __forceinline__ void ry_range(T* re, T* im, int lane, const T* trig, int kbase, T sign = (T)1) {
    if constexpr (Q < QEND) {
        if constexpr (Lay<NQ, HI>::reg(Q) >= 0) {
            const T t = sign * trig[2 * (kbase + Q)], s = sign * trig[2 * (kbase + Q) + 1];
            ry_reg<T, NQ, HI, Q, PAR>(re, im, lane, t, s);
        }
        ry_range<T, NQ, HI, PAR, Q + 1, QEND>(re, im, lane, trig, kbase, sign);
    }
}

template <typename T, int NQ, bool FROM_HI>
__device__ __forceinline__ void relayout(T* re, T* im, cplx<T>* S, int lane) {
    constexpr int R = Lay<NQ, FROM_HI>::R;
#pragma unroll
    for (int r = 0; r < R; ++r) S[pad_slot(Lay<NQ, FROM_HI>::g(lane, r))] = {re[r], im[r]};
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const cplx<T> v = S[pad_slot(Lay<NQ, !FROM_HI>::g(lane, r))];
        re[r] = v.re;
        im[r] = v.im;
    }
    __syncthreads();
}

template <int NQ>
__device__ __forceinline__ bool ladder_flip(int g) {
    constexpr int ladder = (1 << (NQ - 1)) - 1;
    return __popc((unsigned)(g & (g >> 1) & ladder)) & 1;
}

// Write the registers to LDS in natural order, applying S^p (the pending
// CZ-ladder sign) on the way.
template <typename T, int NQ, bool HI>
__device__ __forceinline__ void store_state(const T* re, const T* im, cplx<T>* S, int lane, int p) {
    constexpr int R = Lay<NQ, HI>::R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int g = Lay<NQ, HI>::g(lane, r);
        const bool flip = p && ladder_flip<NQ>(g);
        S[pad_slot(g)] = flip ? cplx<T>{-re[r], -im[r]} : cplx<T>{re[r], im[r]};
    }
    __syncthreads();
}

// Forward pass of the ansatz on the registers (both halves), starting in
// layout LO with p = 0.  Ends in LO (layers even) or HI (odd) with
// p = layers mod 2.
template <typename T, int NQ>
__device__ __forceinline__ void forward_layers(T* re, T* im, cplx<T>* S, const T* trig, int layers,
                                               int lane) {
    int l = 0;
    for (; l + 1 < layers; l += 2) {
        // even layer (p = 0): LO qubits, swap, remaining HI qubits
        ry_range<T, NQ, false, 0, 0, NQ>(re, im, lane, trig, l * NQ);
        relayout<T, NQ, false>(re, im, S, lane);
        ry_range<T, NQ, true, 0, Lay<NQ, false>::RB, NQ>(re, im, lane, trig, l * NQ);
        // odd layer (p = 1): HI qubits, swap, remaining LO qubits
        ry_range<T, NQ, true, 1, 0, NQ>(re, im, lane, trig, (l + 1) * NQ);
        relayout<T, NQ, true>(re, im, S, lane);
        ry_range<T, NQ, false, 1, 0, 5>(re, im, lane, trig, (l + 1) * NQ);
    }
    if (l < layers) {
        ry_range<T, NQ, false, 0, 0, NQ>(re, im, lane, trig, l * NQ);
        relayout<T, NQ, false>(re, im, S, lane);
        ry_range<T, NQ, true, 0, Lay<NQ, false>::RB, NQ>(re, im, lane, trig, l * NQ);
    }
}

// Rotation parameters of every gate: phi = theta/2 reduced to [-pi/2, pi/2].
template <typename T>
__device__ __forceinline__ void rotation_table(const double* __restrict__ theta, int P, T* trig, int lane) {
    for (int k = lane; k < P; k += 64) {
        double ph = 0.5 * theta[k];
        ph -= 3.14159265358979323846 * rint(ph * 0.31830988618379067154);
        trig[2 * k] = (T)tan(0.5 * ph);
        trig[2 * k + 1] = (T)sin(ph);
    }
    __syncthreads();
}

}  // namespace dvq
